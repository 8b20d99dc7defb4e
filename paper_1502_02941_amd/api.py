"""Python binding of libdgdcr.so (include/dgdcr.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch only provides device
memory (tensors) and the current stream.  Importing this module loads the
library and raises if it has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgdcr.so")

DG_OK, DG_NOT_CONVERGED = 0, 1
NIPG, SIPG, IIPG = 1, 2, 3
F64, F32 = 0, 1
DUBINER, MONOMIAL = 0, 1  # element bases (dg_basis)
PART_D, PART_C, PART_R, PART_ALL = 1, 2, 4, 7
ASM_MATRIX_CORE = 256  # parts flag: matrix-core (MFMA) tensor products instead of the vector-ALU kernel (k = 2, 3)
CONST, AFFINE, GAUSS_SUM, QPOINTS = 0, 1, 2, 3
MAX_DEGREE = 4


class DGError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed: %s (%d)" % (what, status_str(status), status))
        self.status = status


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("m", C.c_int32), ("c", C.c_double * 16), ("dev_vals", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("method", C.c_int32), ("degree", C.c_int32), ("sigma", C.c_double), ("sigma_D", C.c_double),
                ("b0", C.c_double), ("eps", _Field), ("bx", _Field), ("by", _Field), ("alpha", _Field),
                ("f", _Field), ("gD", _Field), ("gN", _Field)]


class _MeshInfo(C.Structure):
    _fields_ = [("n_elems", C.c_int64), ("n_int_edges", C.c_int64), ("n_dir_edges", C.c_int64),
                ("n_neu_edges", C.c_int64), ("nnzb", C.c_int64), ("n_dofs", C.c_int64), ("degree", C.c_int32),
                ("n_loc", C.c_int32), ("n_q", C.c_int32), ("n_qe", C.c_int32), ("basis", C.c_int32),
                ("reserved", C.c_int32), ("h_max", C.c_double)]


class _SolverOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iters", C.c_int32), ("rel_tol", C.c_double), ("mixed", C.c_int32),
                ("inner_tol", C.c_double), ("reorth", C.c_int32), ("profile", C.c_int32),
                ("guess_limit", C.c_double), ("persistent", C.c_int32), ("block", C.c_int32),
                ("basis", C.c_int32)]


class _KStats(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double)]


class _Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cycles", C.c_int32), ("reorth_passes", C.c_int32),
                ("rel_res", C.c_double), ("rel_res0", C.c_double), ("guess_rejected", C.c_int32),
                ("persistent", C.c_int32)]


class _Instance(C.Structure):
    _fields_ = [("nodes_xy", C.c_void_p), ("n_nodes", C.c_int64), ("elems", C.c_void_p), ("n_elems", C.c_int64),
                ("dir_edges", C.c_void_p), ("n_dir", C.c_int64), ("neu_edges", C.c_void_p), ("n_neu", C.c_int64),
                ("problem", _Problem)]


class _BatchOpts(C.Structure):
    _fields_ = [("mixed", C.c_int32), ("max_iters", C.c_int32), ("rel_tol", C.c_double), ("inner_tol", C.c_double),
                ("restart_min", C.c_int32), ("restart_max", C.c_int32), ("restart_per_side", C.c_double),
                ("block_threads", C.c_int32), ("slots", C.c_int32), ("lockstep_min_dofs", C.c_int64),
                ("lockstep_mem_gb", C.c_double), ("guess_limit", C.c_double), ("lockstep_block", C.c_int32),
                ("lockstep_eager", C.c_int32), ("lockstep_basis", C.c_int32), ("reserved", C.c_int32)]


class _Reaction(C.Structure):
    _fields_ = [("n", C.c_int32), ("reserved", C.c_int32), ("c", C.c_double * 8)]


class _NewtonOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("reserved", C.c_int32), ("tol", C.c_double)]


class _NewtonReport(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_steps", C.c_int32), ("linear_iters", C.c_int64),
                ("rel_res", C.c_double)]


class _EulerReport(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int32), ("linear_iters", C.c_int64),
                ("newton_steps", C.c_int64), ("rel_res", C.c_double)]


PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32)


REPORT_DTYPE = np.dtype([("status", np.int32), ("iters", np.int32), ("cycles", np.int32), ("reorth", np.int32),
                         ("rel_res", np.float64), ("rel_res0", np.float64), ("guess_rejected", np.int32),
                         ("persistent", np.int32)])

EXPORTS = ["dg_default_penalty", "dg_mesh_create", "dg_mesh_create_basis", "dg_mesh_info_get", "dg_mesh_destroy", "dg_mesh_structure",
           "dg_mesh_qpoints", "dg_assemble", "dg_solver_create", "dg_solver_setup", "dg_solver_solve",
           "dg_solver_destroy", "dg_residual", "dg_status_str", "dg_solver_profile",
           "dg_batch_create", "dg_batch_offsets", "dg_batch_run", "dg_batch_destroy", "dg_batch_progress",
           "dg_batch_set_progress", "dg_mlp_create", "dg_mlp_num_params", "dg_mlp_forward", "dg_mlp_loss_mse",
           "dg_mlp_backward", "dg_mlp_adam_step", "dg_mlp_params", "dg_mlp_destroy", "dg_warmstart_prolong",
           "dg_mesh_error_points", "dg_l2_error", "dg_reaction_terms", "dg_newton_solve", "dg_mesh_refine_sizes",
           "dg_mesh_refine", "dg_implicit_euler", "dg_euler_rhs", "dg_solver_preconditioner", "dg_batch_system",
           "dg_batch_preconditioner", "dg_solve_small_noalloc"]

_lib = None


def lib():
    """Loads libdgdcr.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdgdcr.so is not built (run __graft_entry__.build() or "
                              "python -m paper_1502_02941_amd.build_lib)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.dg_default_penalty.argtypes = [I32, I32, C.POINTER(D), C.POINTER(D)]
        L.dg_mesh_create.argtypes = [P, I64, P, I64, P, I64, P, I64, I32, C.POINTER(P)]
        L.dg_mesh_create_basis.argtypes = [P, I64, P, I64, P, I64, P, I64, I32, I32, C.POINTER(P)]
        L.dg_mesh_info_get.argtypes = [P, C.POINTER(_MeshInfo)]
        L.dg_mesh_destroy.argtypes = [P]
        L.dg_mesh_destroy.restype = None
        L.dg_mesh_structure.argtypes = [P, P, P, P]
        L.dg_mesh_refine_sizes.argtypes = [P, P]
        L.dg_mesh_refine.argtypes = [P, P, P, P, P, P]
        L.dg_mesh_qpoints.argtypes = [P, P, P, P, P, P]
        L.dg_assemble.argtypes = [P, C.POINTER(_Problem), I32, C.c_uint32, P, P, P]
        L.dg_solver_create.argtypes = [P, C.POINTER(_SolverOpts), C.POINTER(P)]
        L.dg_solver_setup.argtypes = [P, P, P]
        L.dg_solver_solve.argtypes = [P, P, P, C.POINTER(_Report), P]
        L.dg_solver_destroy.argtypes = [P]
        L.dg_solver_destroy.restype = None
        L.dg_residual.argtypes = [P, P, P, P, P, P]
        L.dg_solver_profile.argtypes = [P, C.POINTER(_KStats), I32, C.POINTER(I32), I32]
        L.dg_batch_create.argtypes = [C.POINTER(_Instance), I32, C.POINTER(_BatchOpts), C.POINTER(P)]
        L.dg_batch_offsets.argtypes = [P, P]
        L.dg_batch_run.argtypes = [P, P, P, P]
        L.dg_batch_progress.argtypes = [P, C.POINTER(I32)]
        L.dg_batch_set_progress.argtypes = [P, PROGRESS_FN, P]
        L.dg_mlp_create.argtypes = [P, I32, I32, P, C.POINTER(P)]
        L.dg_mlp_num_params.argtypes = [P]
        L.dg_mlp_num_params.restype = I64
        L.dg_mlp_forward.argtypes = [P, P, I32, P, P]
        L.dg_mlp_loss_mse.argtypes = [P, P, I32, P, P, P]
        L.dg_mlp_backward.argtypes = [P, P, I32, P]
        L.dg_mlp_adam_step.argtypes = [P, C.c_float, C.c_float, C.c_float, C.c_float, I32, P]
        L.dg_mlp_params.argtypes = [P, P, P, P]
        L.dg_mlp_destroy.argtypes = [P]
        L.dg_mlp_destroy.restype = None
        L.dg_warmstart_prolong.argtypes = [P, P, I32, I32, I32, P, I64, P]
        L.dg_mesh_error_points.argtypes = [P, P, P]
        L.dg_l2_error.argtypes = [P, P, P, C.POINTER(C.c_double), C.POINTER(C.c_double), P]
        L.dg_reaction_terms.argtypes = [P, C.POINTER(_Reaction), P, P, P, P]
        L.dg_newton_solve.argtypes = [P, C.POINTER(_Reaction), C.POINTER(_NewtonOpts), P, P, P, P,
                                      C.POINTER(_NewtonReport), P]
        L.dg_implicit_euler.argtypes = [P, P, P, P, P, P, D, I32, P, C.POINTER(_EulerReport), P]
        L.dg_euler_rhs.argtypes = [P, P, P, D, P, P]
        L.dg_solver_preconditioner.argtypes = [P, P, P, P]
        L.dg_solve_small_noalloc.argtypes = [P, C.POINTER(_SolverOpts), P, P, P, P, P]
        L.dg_batch_system.argtypes = [P, I32, P, P, P]
        L.dg_batch_preconditioner.argtypes = [P, I32, P, P, P]
        L.dg_batch_destroy.argtypes = [P]
        L.dg_batch_destroy.restype = None
        L.dg_status_str.argtypes = [I32]
        L.dg_status_str.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("dg_mesh_destroy", "dg_solver_destroy", "dg_status_str", "dg_batch_destroy",
                            "dg_mlp_destroy", "dg_mlp_num_params"):
                getattr(L, name).restype = I32
        _lib = L
    return _lib


def status_str(s):
    return lib().dg_status_str(int(s)).decode()


def _check(st, what):
    if st < 0:
        raise DGError(st, what)
    return st


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def default_penalty(method, degree):
    s, k = C.c_double(), C.c_double()
    _check(lib().dg_default_penalty(int(method), int(degree), C.byref(s), C.byref(k)), "dg_default_penalty")
    return s.value, k.value


@dataclass
class Field:
    kind: int = CONST
    c: tuple = (0.0,)
    m: int = 0
    vals: torch.Tensor | None = None

    @staticmethod
    def const(c0):
        return Field(CONST, (float(c0),))

    @staticmethod
    def affine(c0, c1, c2):
        return Field(AFFINE, (float(c0), float(c1), float(c2)))

    @staticmethod
    def gauss_sum(terms):
        flat = tuple(float(v) for t in terms for v in t)
        return Field(GAUSS_SUM, flat, m=len(flat) // 4)

    @staticmethod
    def qpoints(vals: torch.Tensor):
        return Field(QPOINTS, (), vals=vals.contiguous().to(torch.float64))

    def _fill(self, s: _Field):
        s.kind, s.m = int(self.kind), int(self.m)
        for i, v in enumerate(self.c):
            s.c[i] = v
        s.dev_vals = _dptr(self.vals) if self.vals is not None else None


def _as_field(v):
    if v is None:
        return Field.const(0.0)
    return v if isinstance(v, Field) else Field.const(float(v))


@dataclass
class Problem:
    """Data of eq. (1) and the scheme parameters of eq. (ds).  sigma_D <= 0
    selects twice sigma on Dirichlet edges."""
    method: int
    degree: int
    sigma: float
    eps: object
    bx: object
    by: object
    alpha: object
    f: object = None
    gD: object = None
    gN: object = None
    sigma_D: float = 0.0
    b0: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    def _c(self) -> _Problem:
        p = _Problem()
        p.method, p.degree = int(self.method), int(self.degree)
        p.sigma, p.sigma_D, p.b0 = float(self.sigma), float(self.sigma_D), float(self.b0)
        self._keep = []
        for name in ("eps", "bx", "by", "alpha", "f", "gD", "gN"):
            F = _as_field(getattr(self, name))
            self._keep.append(F)
            F._fill(getattr(p, name))
        return p


@dataclass
class RefinedArrays:
    """Device tensors of a refined mesh (dg_mesh_refine); host() gives numpy."""
    nodes: torch.Tensor
    elems: torch.Tensor
    dirichlet: torch.Tensor
    neumann: torch.Tensor

    def host(self):
        return RefinedArrays(*(t.cpu().numpy() for t in (self.nodes, self.elems, self.dirichlet, self.neumann)))


class Mesh:
    """dg_mesh_create_basis on host arrays (0-based; section 2.1 layout);
    basis DUBINER (the paper's default) or MONOMIAL."""

    def __init__(self, nodes, elems, dirichlet, neumann, degree: int, device=None, basis: int = DUBINER):
        if device is not None:
            torch.cuda.set_device(device)
        L = lib()
        if isinstance(nodes, torch.Tensor):
            nodes, elems = nodes.cpu().numpy(), elems.cpu().numpy()
            dirichlet = dirichlet.cpu().numpy() if isinstance(dirichlet, torch.Tensor) else dirichlet
            neumann = neumann.cpu().numpy() if isinstance(neumann, torch.Tensor) else neumann
        nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 2)
        elems = np.ascontiguousarray(elems, dtype=np.int32).reshape(-1, 3)
        d = np.ascontiguousarray(dirichlet if dirichlet is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        nm = np.ascontiguousarray(neumann if neumann is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        h = C.c_void_p()
        st = L.dg_mesh_create_basis(nodes.ctypes.data, len(nodes), elems.ctypes.data, len(elems),
                                    d.ctypes.data if len(d) else None, len(d),
                                    nm.ctypes.data if len(nm) else None, len(nm), int(degree), int(basis), C.byref(h))
        _check(st, "dg_mesh_create_basis")
        self._h = h
        info = _MeshInfo()
        _check(L.dg_mesh_info_get(h, C.byref(info)), "dg_mesh_info_get")
        self.info = {k: getattr(info, k) for k, _ in _MeshInfo._fields_}
        self.T, self.n_loc, self.nnzb, self.n_dofs = info.n_elems, info.n_loc, info.nnzb, info.n_dofs
        self.degree, self.n_q, self.n_qe, self.basis = info.degree, info.n_q, info.n_qe, info.basis
        self.n_bnd = info.n_dir_edges + info.n_neu_edges

    @classmethod
    def from_arrays(cls, m, degree, basis=DUBINER):
        return cls(m.nodes, m.elems, m.dirichlet, m.neumann, degree, basis=basis)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dg_mesh_destroy(h)
            self._h = None

    def refine(self, stream=None):
        """dg_mesh_refine: the uniformly refined mesh arrays as device tensors
        (nodes, elems, dirichlet, neumann), in dg_mesh_create's layout."""
        sz = (C.c_int64 * 4)()
        _check(lib().dg_mesh_refine_sizes(self._h, sz), "dg_mesh_refine_sizes")
        nodes = torch.empty(sz[0], 2, dtype=torch.float64, device="cuda")
        elems = torch.empty(sz[1], 3, dtype=torch.int32, device="cuda")
        d = torch.empty(sz[2], 2, dtype=torch.int32, device="cuda")
        nm = torch.empty(sz[3], 2, dtype=torch.int32, device="cuda")
        _check(lib().dg_mesh_refine(self._h, _dptr(nodes), _dptr(elems), _dptr(d) if sz[2] else None,
                                    _dptr(nm) if sz[3] else None, _stream(stream)), "dg_mesh_refine")
        return RefinedArrays(nodes, elems, d, nm)

    def structure(self, stream=None):
        rp = torch.empty(self.T + 1, dtype=torch.int32, device="cuda")
        ci = torch.empty(self.nnzb, dtype=torch.int32, device="cuda")
        _check(lib().dg_mesh_structure(self._h, _dptr(rp), _dptr(ci), _stream(stream)), "dg_mesh_structure")
        return rp, ci

    def qpoints(self, stream=None):
        vol = torch.empty(self.T, self.n_q, 2, dtype=torch.float64, device="cuda")
        nb = max(self.n_bnd, 1)
        bnd = torch.empty(nb, self.n_qe, 2, dtype=torch.float64, device="cuda")
        nrm = torch.empty(nb, 2, dtype=torch.float64, device="cuda")
        typ = torch.empty(nb, dtype=torch.int32, device="cuda")
        _check(lib().dg_mesh_qpoints(self._h, _dptr(vol), _dptr(bnd), _dptr(nrm), _dptr(typ), _stream(stream)),
               "dg_mesh_qpoints")
        nb = self.n_bnd
        return vol, bnd[:nb], nrm[:nb], typ[:nb]

    def alloc_system(self, prec=F64):
        dt = torch.float64 if prec == F64 else torch.float32
        vals = torch.empty(self.nnzb, self.n_loc, self.n_loc, dtype=dt, device="cuda")
        rhs = torch.empty(self.n_dofs, dtype=dt, device="cuda")
        return vals, rhs


def assemble(mesh: Mesh, prob: Problem, prec=F64, parts=PART_ALL, vals=None, rhs=None, stream=None):
    """dg_assemble into (new or given) tensors; returns (vals, rhs)."""
    if vals is None:
        vals, rhs2 = mesh.alloc_system(prec)
        rhs = rhs2 if rhs is None else rhs
    dt = torch.float64 if prec == F64 else torch.float32
    if vals.dtype != dt or vals.numel() != mesh.nnzb * mesh.n_loc ** 2:
        raise ValueError("vals must hold nnzb*n_loc^2 values of the assembly precision")
    if rhs is not None and (rhs.dtype != dt or rhs.numel() != mesh.n_dofs):
        raise ValueError("rhs must hold n_dofs values of the assembly precision")
    for name, need in (("f", mesh.T * mesh.n_q), ("gD", mesh.n_bnd * mesh.n_qe), ("gN", mesh.n_bnd * mesh.n_qe)):
        F = getattr(prob, name)
        if isinstance(F, Field) and F.kind == QPOINTS and (F.vals is None or F.vals.numel() != need):
            raise ValueError("%s: DG_QPOINTS needs %d device values" % (name, need))
    p = prob._c()
    _check(lib().dg_assemble(mesh._h, C.byref(p), int(prec), int(parts), _dptr(vals), _dptr(rhs), _stream(stream)),
           "dg_assemble")
    return vals, rhs


def residual(mesh: Mesh, vals64, b, x, y=None, stream=None):
    y = torch.empty_like(x) if y is None else y
    _check(lib().dg_residual(mesh._h, _dptr(vals64), _dptr(b), _dptr(x), _dptr(y), _stream(stream)), "dg_residual")
    return y


@dataclass
class Report:
    status: int
    iters: int
    cycles: int
    rel_res: float
    rel_res0: float
    reorth_passes: int = 0
    guess_rejected: int = 0
    persistent: int = 0

    @property
    def converged(self):
        return self.status == DG_OK


class Solver:
    """dg_solver_*: restarted GMRES with right block-Jacobi preconditioning,
    FP64 or FP32 cycles with FP64 refinement (mixed=True)."""

    def __init__(self, mesh: Mesh, restart=50, max_iters=20000, rel_tol=1e-10, mixed=False, inner_tol=1e-5,
                 reorth=False, profile=False, guess_limit=0.0, persistent="auto", block=0, basis=0):
        """persistent: "auto" (one workgroup for small degree-1/2 systems),
        True (always; an error where unsupported) or False (one launch per
        GMRES kernel).  block: Arnoldi vectors per Gram-Schmidt pass of the
        kernel-per-step path (0 automatic: 8, 6 with mixed, 3 above restart 2048; or 1, 2, 3, 4, 6, 8).  basis:
        1 monomial block vectors, 2 shifted by one (0 automatic = 2)."""
        self.mesh = mesh
        pers = {"auto": 0, True: 1, False: -1}[persistent]
        o = _SolverOpts(int(restart), int(max_iters), float(rel_tol), int(bool(mixed)), float(inner_tol),
                        int(bool(reorth)), int(profile), float(guess_limit), pers, int(block), int(basis))
        h = C.c_void_p()
        _check(lib().dg_solver_create(mesh._h, C.byref(o), C.byref(h)), "dg_solver_create")
        self._h = h
        self._vals = None
        self.mixed = bool(mixed)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dg_solver_destroy(h)
            self._h = None

    def setup(self, vals64: torch.Tensor, stream=None):
        assert vals64.dtype == torch.float64
        self._vals = vals64  # the library keeps the pointer: keep the tensor alive
        _check(lib().dg_solver_setup(self._h, _dptr(vals64), _stream(stream)), "dg_solver_setup")

    def profile(self, reset=False):
        """{kernel: (launches, ms, bytes)} from the built-in profiler (profile=True, or 2 for the
        Gram-Schmidt dot kernel alone)."""
        arr = (_KStats * 16)()
        cnt = C.c_int32()
        _check(lib().dg_solver_profile(self._h, arr, 16, C.byref(cnt), int(bool(reset))), "dg_solver_profile")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].bytes) for i in range(cnt.value)}

    def preconditioner(self, stream=None):
        """dg_solver_preconditioner: (D^-1 [T, n, n] FP64, A D^-1 without its
        identity blocks [nnzb - T, n, n] in the cycle precision)."""
        m = self.mesh
        dinv = torch.empty(m.T, m.n_loc, m.n_loc, dtype=torch.float64, device="cuda")
        ahat = torch.empty(max(m.nnzb - m.T, 0), m.n_loc, m.n_loc, dtype=torch.float32 if self.mixed else torch.float64,
                           device="cuda")
        _check(lib().dg_solver_preconditioner(self._h, _dptr(dinv), _dptr(ahat) if ahat.numel() else None,
                                              _stream(stream)), "dg_solver_preconditioner")
        return dinv, ahat

    def solve(self, rhs: torch.Tensor, x: torch.Tensor, stream=None) -> Report:
        r = _Report()
        st = lib().dg_solver_solve(self._h, _dptr(rhs), _dptr(x), C.byref(r), _stream(stream))
        _check(st, "dg_solver_solve")
        return Report(r.status, r.iters, r.cycles, r.rel_res, r.rel_res0, r.reorth_passes, r.guess_rejected,
                      r.persistent)


def solve_small_noalloc(mesh: Mesh, vals64: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor, report: torch.Tensor,
                        restart=50, max_iters=20000, rel_tol=1e-10, mixed=False, inner_tol=1e-5, guess_limit=0.0,
                        stream=None):
    """dg_solve_small_noalloc: setup + one-workgroup GMRES with no allocation;
    report: a device uint8 tensor of REPORT_DTYPE.itemsize bytes (read it with
    Batch.reports)."""
    assert vals64.dtype == torch.float64 and report.numel() == REPORT_DTYPE.itemsize
    o = _SolverOpts(int(restart), int(max_iters), float(rel_tol), int(bool(mixed)), float(inner_tol), 0, 0,
                    float(guess_limit), 1, 1)
    return _check(lib().dg_solve_small_noalloc(mesh._h, C.byref(o), _dptr(vals64), _dptr(rhs), _dptr(x),
                                               _dptr(report), _stream(stream)), "dg_solve_small_noalloc")


def bsr_to_scipy(mesh: Mesh, vals: torch.Tensor, row_ptr=None, col_idx=None):
    """Host copy of the BSR matrix as scipy.sparse.bsr_matrix (for tests and tools)."""
    import scipy.sparse as sp
    if row_ptr is None:
        row_ptr, col_idx = mesh.structure()
    n = mesh.n_loc
    return sp.bsr_matrix((vals.double().cpu().numpy(), col_idx.cpu().numpy(), row_ptr.cpu().numpy()),
                         shape=(mesh.n_dofs, mesh.n_dofs), blocksize=(n, n))


class Batch:
    """dg_batch_*: many independent instances assembled and solved by one
    element-parallel assembly launch and one persistent solve launch.

    instances: list of (MeshArrays, Problem); degree 1 or 2; eps/b/alpha
    CONST or AFFINE, f CONST/AFFINE/GAUSS_SUM, gD/gN CONST/AFFINE."""

    def __init__(self, instances, mixed=True, rel_tol=1e-10, inner_tol=1e-5, max_iters=20000, restart_min=64,
                 restart_per_side=2.0, restart_max=512, block_threads=256, slots=0, lockstep_min_dofs=16384,
                 lockstep_mem_gb=64.0, guess_limit=0.0, log=None, lockstep_block=0, lockstep_eager=False,
                 lockstep_basis=0):
        L = lib()
        self.count = len(instances)
        self.mixed = bool(mixed)
        arr = (_Instance * self.count)()
        self._keep = []
        for i, (m, prob) in enumerate(instances):
            nodes = np.ascontiguousarray(m.nodes, dtype=np.float64)
            el = np.ascontiguousarray(m.elems, dtype=np.int32)
            d = np.ascontiguousarray(m.dirichlet, dtype=np.int32).reshape(-1, 2)
            nm = np.ascontiguousarray(m.neumann, dtype=np.int32).reshape(-1, 2)
            self._keep += [nodes, el, d, nm, prob]
            I = arr[i]
            I.nodes_xy, I.n_nodes = nodes.ctypes.data, len(nodes)
            I.elems, I.n_elems = el.ctypes.data, len(el)
            I.dir_edges, I.n_dir = (d.ctypes.data if len(d) else None), len(d)
            I.neu_edges, I.n_neu = (nm.ctypes.data if len(nm) else None), len(nm)
            I.problem = prob._c()
        o = _BatchOpts(int(bool(mixed)), int(max_iters), float(rel_tol), float(inner_tol), int(restart_min),
                       int(restart_max), float(restart_per_side), int(block_threads), int(slots),
                       int(lockstep_min_dofs), float(lockstep_mem_gb), float(guess_limit), int(lockstep_block),
                       int(lockstep_eager), int(lockstep_basis), 0)
        h = C.c_void_p()
        _check(L.dg_batch_create(arr, self.count, C.byref(o), C.byref(h)), "dg_batch_create")
        self._h = h
        self._log = log
        self._last_progress = [0.0]

        def _progress(user, done, total):
            import time as _t
            now = _t.perf_counter()
            if self._log is not None and (now - self._last_progress[0] >= 20.0 or done == total):
                self._log("batch (lockstep): %d/%d instances finished" % (done, total))
                self._last_progress[0] = now

        self._progress_cb = PROGRESS_FN(_progress)
        _check(L.dg_batch_set_progress(h, self._progress_cb, None), "dg_batch_set_progress")
        self._keep = None
        off = np.zeros(self.count + 1, dtype=np.int64)
        _check(L.dg_batch_offsets(h, off.ctypes.data), "dg_batch_offsets")
        self.offsets = off
        self.n_dofs = int(off[-1])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dg_batch_destroy(h)
            self._h = None

    def alloc(self):
        x = torch.zeros(self.n_dofs, dtype=torch.float64, device="cuda")
        rep = torch.zeros(self.count * REPORT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        return x, rep

    def run(self, x: torch.Tensor, reports: torch.Tensor, stream=None):
        """Asynchronous: assembles and solves every instance (x: initial guesses in, solutions out)."""
        assert x.dtype == torch.float64 and x.numel() == self.n_dofs
        assert reports.numel() == self.count * REPORT_DTYPE.itemsize
        _check(lib().dg_batch_run(self._h, _dptr(x), _dptr(reports), _stream(stream)), "dg_batch_run")

    def progress(self):
        """Instances started by the running (or last) launch."""
        v = C.c_int32()
        _check(lib().dg_batch_progress(self._h, C.byref(v)), "dg_batch_progress")
        return v.value

    def wait(self, log=None, every=20.0, stream=None):
        """Waits for the launch, printing the number of started instances when it
        changes (at most every `every` seconds)."""
        import time as _t
        ev = torch.cuda.Event()
        ev.record(stream if stream is not None else torch.cuda.current_stream())
        last_t, last_v = _t.perf_counter(), -1
        while not ev.query():
            _t.sleep(0.05)
            now = _t.perf_counter()
            if log and now - last_t >= every:
                v = self.progress()
                if v != last_v:
                    log("batch: %d/%d instances started" % (v, self.count))
                    last_v = v
                last_t = now
        ev.synchronize()

    def system(self, i, n_loc, nnzb, stream=None):
        """dg_batch_system: FP64 BSR values [nnzb, n_loc, n_loc] and load vector of instance i."""
        n = int(self.offsets[i + 1] - self.offsets[i])
        vals = torch.empty(nnzb, n_loc, n_loc, dtype=torch.float64, device="cuda")
        rhs = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().dg_batch_system(self._h, int(i), _dptr(vals), _dptr(rhs), _stream(stream)), "dg_batch_system")
        return vals, rhs

    def preconditioner(self, i, n_loc, nnzb, stream=None):
        """dg_batch_preconditioner: (D^-1 FP64, A D^-1 off-diagonal blocks in the cycle precision) of instance i."""
        T = int(self.offsets[i + 1] - self.offsets[i]) // n_loc
        dinv = torch.empty(T, n_loc, n_loc, dtype=torch.float64, device="cuda")
        ahat = torch.empty(max(nnzb - T, 1), n_loc, n_loc, dtype=torch.float32 if self.mixed else torch.float64,
                           device="cuda")
        _check(lib().dg_batch_preconditioner(self._h, int(i), _dptr(dinv), _dptr(ahat), _stream(stream)),
               "dg_batch_preconditioner")
        return dinv, ahat[:max(nnzb - T, 0)]

    @staticmethod
    def reports(rep: torch.Tensor):
        return np.frombuffer(rep.cpu().numpy().tobytes(), dtype=REPORT_DTYPE)

    def segment(self, x, i):
        return x[int(self.offsets[i]):int(self.offsets[i + 1])]


def instance_problem(inst, method=SIPG):
    """Problem of a sampled batch instance (workloads.Instance): SIPG with the
    default penalty, constant eps, b, alpha, Gaussian-sum f, g^D = 0."""
    sigma, _ = default_penalty(method, inst.k)
    bx, by = inst.b
    return Problem(method, inst.k, sigma, eps=inst.eps, bx=bx, by=by, alpha=inst.alpha,
                   f=Field.gauss_sum([tuple(t) for t in inst.gauss]), gD=0.0)


class MLP:
    """dg_mlp_*: the perceptron of the learned initial guess (BF16 products,
    FP32 accumulation and master weights, Adam)."""

    def __init__(self, widths, max_batch, init_params):
        L = lib()
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        p0 = np.ascontiguousarray(init_params, dtype=np.float32)
        w = np.asarray(self.widths, dtype=np.int32)
        h = C.c_void_p()
        _check(L.dg_mlp_create(w.ctypes.data, len(w), self.max_batch, p0.ctypes.data, C.byref(h)), "dg_mlp_create")
        self._h = h
        self.n_params = int(L.dg_mlp_num_params(h))
        assert self.n_params == p0.size, "init_params has the wrong length"
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.t = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.dg_mlp_destroy(h)
            self._h = None

    def forward(self, x: torch.Tensor, y: torch.Tensor = None, stream=None):
        x = x.contiguous().float()
        B = x.shape[0]
        if y is None:
            y = torch.empty(B, self.widths[-1], dtype=torch.float32, device="cuda")
        _check(lib().dg_mlp_forward(self._h, _dptr(x), B, _dptr(y), _stream(stream)), "dg_mlp_forward")
        return y

    def loss_mse(self, target: torch.Tensor, stream=None):
        target = target.contiguous().float()
        dy = torch.empty_like(target)
        _check(lib().dg_mlp_loss_mse(self._h, _dptr(target), target.shape[0], _dptr(dy), _dptr(self._loss),
                                     _stream(stream)), "dg_mlp_loss_mse")
        return self._loss, dy

    def backward(self, dy: torch.Tensor, stream=None):
        dy = dy.contiguous().float()
        _check(lib().dg_mlp_backward(self._h, _dptr(dy), dy.shape[0], _stream(stream)), "dg_mlp_backward")

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.t += 1
        _check(lib().dg_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), self.t,
                                      _stream(stream)), "dg_mlp_adam_step")

    def params(self, stream=None):
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().dg_mlp_params(self._h, _dptr(p), _dptr(g), _stream(stream)), "dg_mlp_params")
        return p, g


def warmstart_prolong(mesh: Mesh, coarse: torch.Tensor, nc: int, mode: int, x: torch.Tensor, stream=None):
    """dg_warmstart_prolong: coarse [B, nc*nc] FP32 -> x [B, ldx] FP64 (mode 0 injection, 1 bilinear P1)."""
    coarse = coarse.contiguous().float()
    assert x.dtype == torch.float64 and x.dim() == 2 and x.is_contiguous()
    _check(lib().dg_warmstart_prolong(mesh._h, _dptr(coarse), coarse.shape[0], int(nc), int(mode), _dptr(x),
                                      x.shape[1], _stream(stream)), "dg_warmstart_prolong")
    return x


def error_points(mesh: Mesh, stream=None):
    """dg_mesh_error_points: [T, (k+4)^2, 2] physical points of the error rule."""
    q = mesh.info["degree"] + 4
    out = torch.empty(mesh.T, q * q, 2, dtype=torch.float64, device="cuda")
    _check(lib().dg_mesh_error_points(mesh._h, _dptr(out), _stream(stream)), "dg_mesh_error_points")
    return out


def l2_error(mesh: Mesh, x: torch.Tensor, exact, stream=None):
    """dg_l2_error: (||u_h - u||_L2, h_max).  exact: values at error_points()
    ([T, (k+4)^2] FP64 tensor) or a function u(x, y) of numpy arrays."""
    if callable(exact):
        pts = error_points(mesh, stream).cpu().numpy()
        exact = torch.from_numpy(np.ascontiguousarray(exact(pts[..., 0], pts[..., 1]), dtype=np.float64)).cuda()
    exact = exact.contiguous().to(torch.float64)
    l2, hmax = C.c_double(), C.c_double()
    _check(lib().dg_l2_error(mesh._h, _dptr(x), _dptr(exact), C.byref(l2), C.byref(hmax), _stream(stream)),
           "dg_l2_error")
    return l2.value, hmax.value


def _reaction(c):
    c = [float(v) for v in c]
    if len(c) > 8:
        raise ValueError("at most 8 reaction terms")
    r = _Reaction()
    r.n = len(c)
    for i, v in enumerate(c):
        r.c[i] = v
    return r


def reaction_terms(mesh: Mesh, c, x: torch.Tensor, stream=None):
    """dg_reaction_terms: H(x) [n_dofs] and the Jacobian's diagonal blocks HJ
    [T, n_loc, n_loc] for r(u) = sum_p c[p-1] u^p."""
    r = _reaction(c)
    h = torch.empty(mesh.n_dofs, dtype=torch.float64, device="cuda")
    hj = torch.empty(mesh.T, mesh.n_loc, mesh.n_loc, dtype=torch.float64, device="cuda")
    _check(lib().dg_reaction_terms(mesh._h, C.byref(r), _dptr(x), _dptr(h), _dptr(hj), _stream(stream)),
           "dg_reaction_terms")
    return h, hj


def newton_solve(mesh: Mesh, solver, vals64: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor, c, tol=1e-10,
                 max_newton=50, stream=None):
    """dg_newton_solve: Newton's method for (D + C + R) v + H(v) = F; x holds
    the initial guess and receives the solution.  The solver must be set up
    again before its next plain solve."""
    r = _reaction(c)
    o = _NewtonOpts(int(max_newton), 0, float(tol))
    rep = _NewtonReport()
    st = lib().dg_newton_solve(mesh._h, C.byref(r), C.byref(o), solver._h, _dptr(vals64), _dptr(rhs), _dptr(x),
                               C.byref(rep), _stream(stream))
    _check(st, "dg_newton_solve")
    return {"status": rep.status, "newton_steps": rep.newton_steps, "linear_iters": rep.linear_iters,
            "rel_res": rep.rel_res}


def euler_rhs(mesh: Mesh, rhs: torch.Tensor, u: torch.Tensor, inv_dt: float, out=None, stream=None):
    """dg_euler_rhs: rhs + inv_dt M u (M the mass matrix)."""
    if out is None:
        out = torch.empty_like(rhs)
    _check(lib().dg_euler_rhs(mesh._h, _dptr(rhs), _dptr(u), float(inv_dt), _dptr(out), _stream(stream)),
           "dg_euler_rhs")
    return out


def implicit_euler(mesh: Mesh, solver, vals64: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor, inv_dt: float,
                   n_steps: int, c=None, tol=1e-10, max_newton=50, stream=None):
    """dg_implicit_euler: n_steps backward Euler steps from x = u^0 (x receives
    u^n).  vals64 is assembled with alpha = alpha_0 + inv_dt; c (optional) are
    the coefficients of the non-linear reaction r(u) = sum_p c[p-1] u^p, each
    step then solved by Newton's method with tolerance tol."""
    rep = _EulerReport()
    if c is None:
        st = lib().dg_implicit_euler(mesh._h, None, None, solver._h, _dptr(vals64), _dptr(rhs), float(inv_dt),
                                     int(n_steps), _dptr(x), C.byref(rep), _stream(stream))
    else:
        r = _reaction(c)
        o = _NewtonOpts(int(max_newton), 0, float(tol))
        st = lib().dg_implicit_euler(mesh._h, C.byref(r), C.byref(o), solver._h, _dptr(vals64), _dptr(rhs),
                                     float(inv_dt), int(n_steps), _dptr(x), C.byref(rep), _stream(stream))
    _check(st, "dg_implicit_euler")
    return {"status": rep.status, "steps": rep.steps, "linear_iters": rep.linear_iters,
            "newton_steps": rep.newton_steps, "rel_res": rep.rel_res}
