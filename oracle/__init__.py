"""Oracle for the DG diffusion-convection-reaction method -- TEST INFRASTRUCTURE.

A plain FP64 CPU implementation (``dg_oracle.c``) of the discretisation of
Uzunca & Karasozen (arXiv:1502.02941): the interior-penalty bilinear form a_h
and load functional l_h of section 1, eq. (ds), split into the diffusion,
convection and reaction matrices D, C, R and the vector F of section 2.3,
eqs. (dgscheme) and (system), plus a plain restarted GMRES with a right
block-Jacobi preconditioner and the L2 error of section 2.4.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library and imports nothing from it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The mutation tests point this at a deliberately broken copy of the oracle.
_LIB_OVERRIDE = os.environ.get("DG_ORACLE_LIB")

PART_D, PART_C, PART_R = 1, 2, 4
PART_ALL = PART_D | PART_C | PART_R
CONST, AFFINE, GAUSS_SUM, POINTS = 0, 1, 2, 3
NIPG, SIPG, IIPG = 1, 2, 3  # the paper's method numbering (section 2.2)


def build(force: bool = True) -> str:
    """Compile dg_oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=True)
            L = C.CDLL(_LIB)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_mesh_create.argtypes = [P, I64, P, I64, P, I64, P, I64, C.POINTER(P)]
        L.orc_mesh_create.restype = C.c_int
        L.orc_mesh_free.argtypes = [P]
        L.orc_mesh_counts.argtypes = [P, P]
        L.orc_mesh_counts.restype = I64
        L.orc_mesh_hmax.argtypes = [P]
        L.orc_mesh_hmax.restype = D
        L.orc_mesh_edges.argtypes = [P, P, P, P, P, P]
        L.orc_volume_rule.argtypes = [C.c_int, P, P, P]
        L.orc_edge_rule.argtypes = [C.c_int, P, P]
        L.orc_basis_eval.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P]
        L.orc_volume_points.argtypes = [P, C.c_int, C.c_int, P]
        L.orc_boundary_points.argtypes = [P, C.c_int, P, P]
        L.orc_assemble.argtypes = [P, P, C.c_uint32, P, P, P, P]
        L.orc_assemble.restype = C.c_int
        L.orc_matvec.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_gmres.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int, D, C.c_int,
                                C.POINTER(C.c_int), C.POINTER(D)]
        L.orc_gmres.restype = C.c_int
        L.orc_eval_solution.argtypes = [P, C.c_int, C.c_int, P, I64, P, P, P]
        L.orc_eval_solution.restype = C.c_int
        L.orc_l2_error.argtypes = [P, C.c_int, C.c_int, P, C.c_int, P]
        L.orc_l2_error.restype = D
        L.orc_reaction_terms.argtypes = [P, C.c_int, C.c_int, C.c_int, P, P, P, P]
        L.orc_reaction_terms.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    pass


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("c", C.c_double * 16), ("vals", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("degree", C.c_int32), ("basis", C.c_int32), ("sigma", C.c_double), ("sigma_D", C.c_double),
                ("kappa", C.c_double), ("b0", C.c_double),
                ("eps", _Field), ("bx", _Field), ("by", _Field), ("alpha", _Field),
                ("f", _Field), ("gD", _Field), ("gN", _Field)]


class Field:
    """A coefficient or data field: CONST c0, AFFINE c0 + c1 x + c2 y,
    GAUSS_SUM sum_m A_m exp(-|x - c_m|^2 / (2 w_m^2)), or POINTS (values at the
    oracle's own quadrature points, see volume_points / boundary_points)."""

    def __init__(self, kind, c=(), m=0, vals=None):
        self.kind, self.c, self.m = kind, tuple(float(v) for v in c), m
        self.vals = None if vals is None else np.ascontiguousarray(vals, dtype=np.float64)

    @staticmethod
    def const(c0):
        return Field(CONST, (c0,))

    @staticmethod
    def affine(c0, c1, c2):
        return Field(AFFINE, (c0, c1, c2))

    @staticmethod
    def gauss_sum(terms):
        """terms: iterable of (cx, cy, width, amplitude)."""
        flat = [float(v) for t in terms for v in t]
        return Field(GAUSS_SUM, flat, m=len(flat) // 4)

    @staticmethod
    def points(vals):
        return Field(POINTS, (), vals=vals)

    def _fill(self, s: _Field):
        s.kind, s.m = self.kind, self.m
        for i, v in enumerate(self.c):
            s.c[i] = v
        s.vals = _ptr(self.vals) if self.vals is not None else None


def default_penalty(method: int, k: int):
    """(sigma, kappa) of the paper's set_parameter table (section 4): NIPG kappa=+1,
    sigma=1; SIPG kappa=-1, sigma=3k(k+1); IIPG kappa=0, sigma=3k(k+1)."""
    if method == NIPG:
        return 1.0, 1.0
    if method == SIPG:
        return 3.0 * k * (k + 1), -1.0
    if method == IIPG:
        return 3.0 * k * (k + 1), 0.0
    raise OracleError("unknown method %r" % (method,))


class Mesh:
    """The oracle's mesh: element connectivity plus interior / Dirichlet /
    Neumann edge classification (section 2.1).  Inputs are 0-based."""

    def __init__(self, nodes, elems, dirichlet=None, neumann=None):
        L = lib()
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 2)
        self.elems = np.ascontiguousarray(elems, dtype=np.int32).reshape(-1, 3)
        d = np.ascontiguousarray(dirichlet if dirichlet is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        nm = np.ascontiguousarray(neumann if neumann is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        h = C.c_void_p()
        st = L.orc_mesh_create(_ptr(self.nodes), len(self.nodes), _ptr(self.elems), len(self.elems),
                               _ptr(d), len(d), _ptr(nm), len(nm), C.byref(h))
        if st != 0:
            raise OracleError("orc_mesh_create failed with status %d" % st)
        self._h = h
        cnt = np.zeros(6, dtype=np.int64)
        L.orc_mesh_counts(h, _ptr(cnt))
        self.T, self.n_int, self.n_bnd, self.n_dir, self.n_neu = (int(v) for v in cnt[:5])
        self.int_el = np.zeros((self.n_int, 2), dtype=np.int32)
        self.int_v = np.zeros((self.n_int, 2), dtype=np.int32)
        self.bnd_el = np.zeros(self.n_bnd, dtype=np.int32)
        self.bnd_v = np.zeros((self.n_bnd, 2), dtype=np.int32)
        self.bnd_type = np.zeros(self.n_bnd, dtype=np.int32)
        L.orc_mesh_edges(h, _ptr(self.int_el), _ptr(self.int_v), _ptr(self.bnd_el), _ptr(self.bnd_v),
                         _ptr(self.bnd_type))
        self.hmax = float(L.orc_mesh_hmax(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_mesh_free(h)
            self._h = None

    def volume_points(self, q):
        out = np.zeros((self.T, q * q, 2))
        lib().orc_volume_points(self._h, 0, q, _ptr(out))
        return out

    def boundary_points(self, q):
        out = np.zeros((self.n_bnd, q, 2))
        nrm = np.zeros((self.n_bnd, 2))
        lib().orc_boundary_points(self._h, q, _ptr(out), _ptr(nrm))
        return out, nrm


def volume_rule(q):
    xi, eta, w = np.zeros(q * q), np.zeros(q * q), np.zeros(q * q)
    lib().orc_volume_rule(q, _ptr(xi), _ptr(eta), _ptr(w))
    return xi, eta, w


def edge_rule(q):
    t, w = np.zeros(q), np.zeros(q)
    lib().orc_edge_rule(q, _ptr(t), _ptr(w))
    return t, w


# Element bases: the orthonormal Dubiner basis (the paper's default, base = 2
# of set_parameter) and monomials xi^p eta^q in the same order (base = 1).
DUBINER, MONOMIAL = 0, 1


def basis_eval(k, xi, eta, basis=DUBINER):
    """Basis values and reference gradients, each [npts][n_loc]."""
    xi = np.ascontiguousarray(xi, dtype=np.float64).ravel()
    eta = np.ascontiguousarray(eta, dtype=np.float64).ravel()
    n = (k + 1) * (k + 2) // 2
    v, dx, de = (np.zeros((len(xi), n)) for _ in range(3))
    r = lib().orc_basis_eval(k, basis, len(xi), _ptr(xi), _ptr(eta), _ptr(v), _ptr(dx), _ptr(de))
    if r < 0:
        raise OracleError("bad degree or basis")
    return v, dx, de


class Blocks:
    """Assembled system: diagonal blocks, the two off-diagonal blocks of every
    interior edge, and the load vector."""

    def __init__(self, mesh, k, diag, off_ij, off_ji, rhs, basis=DUBINER):
        self.mesh, self.k, self.basis = mesh, k, basis
        self.n = (k + 1) * (k + 2) // 2
        self.diag, self.off_ij, self.off_ji, self.rhs = diag, off_ij, off_ji, rhs

    def to_scipy(self):
        import scipy.sparse as sp
        n, M = self.n, self.mesh
        rows, cols, vals = [], [], []
        ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        K = np.arange(M.T)
        rows.append((K[:, None, None] * n + ii[None]).ravel())
        cols.append((K[:, None, None] * n + jj[None]).ravel())
        vals.append(self.diag.ravel())
        Ki, Kj = M.int_el[:, 0].astype(np.int64), M.int_el[:, 1].astype(np.int64)
        rows.append((Ki[:, None, None] * n + ii[None]).ravel())
        cols.append((Kj[:, None, None] * n + jj[None]).ravel())
        vals.append(self.off_ij.ravel())
        rows.append((Kj[:, None, None] * n + ii[None]).ravel())
        cols.append((Ki[:, None, None] * n + jj[None]).ravel())
        vals.append(self.off_ji.ravel())
        N = M.T * n
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))

    def matvec(self, x):
        y = np.zeros(self.mesh.T * self.n)
        x = np.ascontiguousarray(x, dtype=np.float64)
        lib().orc_matvec(self.mesh._h, self.k, _ptr(self.diag), _ptr(self.off_ij), _ptr(self.off_ji),
                         _ptr(x), _ptr(y))
        return y

    def block(self, row_el, col_el):
        """The n x n block (row element, column element), zero if not coupled."""
        if row_el == col_el:
            return self.diag[row_el]
        M = self.mesh
        for e in range(M.n_int):
            a, b = M.int_el[e]
            if a == row_el and b == col_el:
                return self.off_ij[e]
            if b == row_el and a == col_el:
                return self.off_ji[e]
        return np.zeros((self.n, self.n))


def assemble(mesh: Mesh, k: int, *, sigma, kappa, eps, bx, by, alpha, f, gD=None, gN=None,
             sigma_D=None, b0=1.0, parts=PART_ALL, basis=DUBINER) -> Blocks:
    """Assemble D+C+R (parts selected by the bit mask) and F.  Scalar arguments
    are promoted to CONST fields.  sigma_D defaults to 2*sigma (section 1)."""

    def fld(v):
        if v is None:
            return Field.const(0.0)
        return v if isinstance(v, Field) else Field.const(v)

    P = _Problem()
    P.degree = k
    P.basis = basis
    P.sigma = float(sigma)
    P.sigma_D = float(2.0 * sigma if sigma_D is None else sigma_D)
    P.kappa = float(kappa)
    P.b0 = float(b0)
    keep = []
    for name, v in (("eps", eps), ("bx", bx), ("by", by), ("alpha", alpha), ("f", f), ("gD", gD), ("gN", gN)):
        F = fld(v)
        keep.append(F)
        F._fill(getattr(P, name))
    n = (k + 1) * (k + 2) // 2
    if f is not None and isinstance(f, Field) and f.kind == POINTS:
        assert f.vals.size == mesh.T * (k + 2) ** 2, "f POINTS must match volume_points(k+2)"
    for g in (gD, gN):
        if isinstance(g, Field) and g.kind == POINTS:
            assert g.vals.size == mesh.n_bnd * (k + 2), "boundary POINTS must match boundary_points(k+2)"
    diag = np.zeros((mesh.T, n, n))
    off_ij = np.zeros((mesh.n_int, n, n))
    off_ji = np.zeros((mesh.n_int, n, n))
    rhs = np.zeros(mesh.T * n)
    st = lib().orc_assemble(mesh._h, C.byref(P), parts, _ptr(diag), _ptr(off_ij), _ptr(off_ji), _ptr(rhs))
    if st != 0:
        raise OracleError("orc_assemble failed with status %d" % st)
    return Blocks(mesh, k, diag, off_ij, off_ji, rhs, basis)


def gmres(blocks: Blocks, rhs=None, x0=None, restart=50, tol=1e-10, max_iters=100000):
    """Right block-Jacobi preconditioned GMRES(restart).  Returns (x, iters, relres, converged)."""
    M = blocks.mesh
    F = np.ascontiguousarray(blocks.rhs if rhs is None else rhs, dtype=np.float64)
    x = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.float64)
    its, rel = C.c_int(0), C.c_double(0.0)
    st = lib().orc_gmres(M._h, blocks.k, _ptr(blocks.diag), _ptr(blocks.off_ij), _ptr(blocks.off_ji),
                         _ptr(F), _ptr(x), int(restart), float(tol), int(max_iters), C.byref(its), C.byref(rel))
    if st < 0:
        raise OracleError("orc_gmres failed with status %d" % st)
    return x, its.value, rel.value, st == 0


def eval_solution(mesh: Mesh, k: int, coef, elem, xy, basis=DUBINER):
    elem = np.ascontiguousarray(elem, dtype=np.int32)
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    out = np.zeros(len(elem))
    if lib().orc_eval_solution(mesh._h, k, basis, _ptr(coef), len(elem), _ptr(elem), _ptr(xy), _ptr(out)) != 0:
        raise OracleError("orc_eval_solution: bad degree or basis")
    return out


def l2_error(mesh: Mesh, k: int, coef, exact_fn, q=None, basis=DUBINER):
    """||u_h - u||_L2 with a Stroud rule of q (default k+4) points per direction;
    exact_fn(x, y) is evaluated at the oracle's own points."""
    q = k + 4 if q is None else q
    pts = mesh.volume_points(q)
    ex = np.ascontiguousarray(exact_fn(pts[..., 0], pts[..., 1]), dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    return float(lib().orc_l2_error(mesh._h, k, basis, _ptr(coef), q, _ptr(ex)))


# ----------------------------------------------------------------------------
# Non-linear reaction and Newton's method (section 3).
# ----------------------------------------------------------------------------
def reaction_terms(mesh: Mesh, k: int, c, coef, basis=DUBINER):
    """H_i = int r(u_h) phi_i and the diagonal blocks HJ[K] (row = test) of its
    Jacobian, r(u) = sum_p c[p-1] u^p, with the assembly's volume rule."""
    n = (k + 1) * (k + 2) // 2
    c = np.ascontiguousarray(c, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    h = np.zeros(mesh.T * n)
    hj = np.zeros((mesh.T, n, n))
    st = lib().orc_reaction_terms(mesh._h, k, basis, len(c), _ptr(c), _ptr(coef), _ptr(h), _ptr(hj))
    if st != 0:
        raise OracleError("orc_reaction_terms: %d" % st)
    return h, hj


def newton(mesh: Mesh, k: int, blocks, c, tol=1e-10, max_newton=50, x0=None, rhs=None):
    """Newton's method for (D + C + R) v + H(v) = F: J w = -Res, v <- v + w with
    Res = A v + H(v) - F and J = A + HJ(v); every linear system is solved
    directly.  Stops when ||Res|| / ||F|| <= tol (checked before each step).
    F is blocks.rhs unless rhs is given.
    Returns (v, newton steps, final relative residual, converged)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    A = blocks.to_scipy().tocsr()
    F = blocks.rhs if rhs is None else np.asarray(rhs, dtype=np.float64)
    n = (k + 1) * (k + 2) // 2
    T = mesh.T
    x = np.zeros(T * n) if x0 is None else np.array(x0, dtype=np.float64)
    fn = np.linalg.norm(F)
    rel = np.inf
    for it in range(max_newton + 1):
        h, hj = reaction_terms(mesh, k, c, x, basis=blocks.basis)
        res = A @ x + h - F
        rel = np.linalg.norm(res) / fn
        if rel <= tol:
            return x, it, rel, True
        if it == max_newton:
            break
        HJ = sp.bsr_matrix((hj, np.arange(T), np.arange(T + 1)), shape=(T * n, T * n))
        x = x + spl.spsolve((A + HJ).tocsc(), -res)
    return x, max_newton, rel, False


def uniform_refine(nodes, elems, dirichlet, neumann):
    """Red refinement of a triangulation (the refinement step of the paper's
    driver, section 2.1), in plain Python: each triangle (a, b, c) is cut at its
    edge midpoints into (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca),
    and each listed boundary edge (a, b) into (a, m), (m, b).  A midpoint is a
    new node numbered after the existing ones in the order the edges are first
    met when the triangles are visited in order, each through its edges
    (a, b), (b, c), (c, a).  Returns (nodes, elems, dirichlet, neumann)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    new_nodes = [list(p) for p in nodes]
    index_of = {}

    def mid(a, b):
        e = frozenset((int(a), int(b)))
        if e not in index_of:
            index_of[e] = len(new_nodes)
            new_nodes.append([0.5 * (nodes[a][0] + nodes[b][0]), 0.5 * (nodes[a][1] + nodes[b][1])])
        return index_of[e]

    tris = []
    for a, b, c in np.asarray(elems):
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        tris += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]

    def halves(edges):
        out = []
        for a, b in np.asarray(edges).reshape(-1, 2):
            m = index_of[frozenset((int(a), int(b)))]
            out += [[a, m], [m, b]]
        return np.array(out, dtype=np.int32).reshape(-1, 2)

    return (np.array(new_nodes, dtype=np.float64), np.array(tris, dtype=np.int32), halves(dirichlet),
            halves(neumann))


def implicit_euler(mesh: Mesh, k: int, blocks, mass, inv_dt, n_steps, x0=None, c=None, tol=1e-10, max_newton=50):
    """Backward Euler: section 3 reads its linear reaction coefficient as 1/dt
    of a time discretisation.  `blocks` holds D + C + R assembled with
    alpha = alpha_0 + inv_dt and F; `mass` the mass matrix (R assembled with
    alpha = 1).  Each step solves A u^{n+1} [+ H(u^{n+1})] = F + inv_dt M u^n
    directly (by Newton's method from u^n when c is given).  Returns u^n_steps."""
    import scipy.sparse.linalg as spl
    A = blocks.to_scipy().tocsc()
    M = mass.to_scipy().tocsr()
    x = np.zeros(A.shape[0]) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(n_steps):
        rhs = blocks.rhs + inv_dt * (M @ x)
        if c is None:
            x = spl.spsolve(A, rhs)
        else:
            x, _, _, ok = newton(mesh, k, blocks, c, tol=tol, max_newton=max_newton, x0=x, rhs=rhs)
            if not ok:
                raise OracleError("implicit_euler: Newton did not converge")
    return x
