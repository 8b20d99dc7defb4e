/*
 * dgdcr.h -- C ABI of the MI355X (gfx950) discontinuous Galerkin library for
 * steady diffusion-convection-reaction problems
 *
 *     alpha u - eps Lap u + b . grad u = f   in Omega,
 *     u = g^D on Gamma^D,   eps grad u . n = g^N on Gamma^N,
 *
 * discretised as in Uzunca & Karasozen, "A Matlab Tutorial for
 * Diffusion-Convection-Reaction Equations using DGFEM" (arXiv:1502.02941),
 * section 1 eq. (1) and the interior penalty scheme eq. (ds): SIPG / NIPG /
 * IIPG diffusion, upwind convection, reaction, and the load functional l_h.
 * The matrix is D + C + R of section 2.3 eq. (dgscheme) and (system) in
 * block-sparse row (BSR) form; it is solved by restarted GMRES with a right
 * block-Jacobi preconditioner, in FP64 or with FP32 Arnoldi cycles and FP64
 * residual / update steps (iterative refinement).
 *
 * Conventions shared by every call:
 *  - indices are 0-based (the paper's arrays are 1-based);
 *  - "dev_" pointers are device (HIP) memory owned by the caller; "host"
 *    pointers are host memory owned by the caller and only read during the
 *    call; objects (dg_mesh, dg_solver) are owned by the library until their
 *    _destroy call;
 *  - `stream` is a hipStream_t (NULL = the default stream); device work is
 *    stream-ordered and the call returns before it finishes unless stated;
 *  - errors are returned as negative dg_status codes, never by aborting;
 *    a positive code is a warning (the outputs are valid but see the code).
 *
 * Layouts:
 *  - element-local basis: orthonormal Dubiner basis of degree k on the
 *    reference triangle (the paper's default, base = 2 of set_parameter), or
 *    with dg_mesh_create_basis the monomials xi^p eta^q (base = 1); either way
 *    n_loc = (k+1)(k+2)/2 functions ordered by total degree d = 0..k, then
 *    q = 0..d (p = d-q); vertex 1 of an element row maps to (0,0), vertex 2
 *    to (1,0), vertex 3 to (0,1);
 *  - dof index = element * n_loc + local index (element-major);
 *  - BSR: row_ptr[T+1], col_idx[nnzb] (int32); block row K holds the
 *    diagonal block first, then one block per interior neighbour in local
 *    edge order (edge l joins vertex l and vertex l+1 mod 3); values are
 *    [nnzb][n_loc][n_loc] row-major, row = test function phi_i, column =
 *    trial function phi_j (entry = a_h(phi_j, phi_i)), FP64 or FP32.
 */
#ifndef DGDCR_H
#define DGDCR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DG_OK = 0,
    DG_NOT_CONVERGED = 1,       /* warning: iteration cap reached; x holds the last iterate */
    DG_ERR_ARG = -1,            /* null pointer, size or enum out of range, degree mismatch */
    DG_ERR_ORIENTATION = -2,    /* an element is not counter-clockwise (det J <= 0), section 2.1 */
    DG_ERR_BOUNDARY = -3,       /* a boundary edge is not listed in exactly one of Dirichlet /
                                   Neumann, or a listed edge is not a boundary edge (eq. 1) */
    DG_ERR_NONMANIFOLD = -4,    /* an edge shared by more than two elements, or a repeated element */
    DG_ERR_DEGREE = -5,         /* degree outside [0, DG_MAX_DEGREE], or sigma undefined for k = 0 */
    DG_ERR_METHOD = -6,         /* method not NIPG / SIPG / IIPG */
    DG_ERR_NONFINITE = -7,      /* NaN / Inf in coordinates, parameters or a residual norm */
    DG_ERR_HIP = -8,            /* a HIP runtime call failed */
    DG_ERR_OOM = -9             /* device or host allocation failed */
} dg_status;

#define DG_MAX_DEGREE 4

/* Method numbering of the paper's set_parameter routine (section 2.2, section 4). */
typedef enum { DG_NIPG = 1, DG_SIPG = 2, DG_IIPG = 3 } dg_method;
typedef enum { DG_F64 = 0, DG_F32 = 1 } dg_prec;
/* Element basis (section 4, set_parameter's `base`): 2 there is the
 * orthonormal Dubiner basis, 1 the monomials. */
typedef enum { DG_BASIS_DUBINER = 0, DG_BASIS_MONOMIAL = 1 } dg_basis;

/* Parts of a_h = D_h + C_h + R_h (section 2.3 eq. (dgscheme)) selected by dg_assemble. */
enum { DG_PART_D = 1, DG_PART_C = 2, DG_PART_R = 4, DG_PART_ALL = 7 };
/* Added to `parts`: with degree 2 or 3 and constant eps and alpha, assemble the
 * blocks of 16 elements at a time as matrix-core (MFMA) products of their
 * coefficient rows with the reference tensors (two launches: coefficients, then
 * products) instead of with the default vector-ALU tensor kernel (one lane per
 * element and trial function).  Both compute the same terms; the results differ
 * by rounding only.  The matrix-core path keeps a [47][n_elems] FP64-sized
 * coefficient array in the mesh, allocated by its first call (DG_ERR_OOM if
 * that fails): dg_assemble calls on one mesh that overlap in time must not both
 * use it.  Ignored for other degrees and for variable eps or alpha. */
enum { DG_ASM_MATRIX_CORE = 256 };

/* A coefficient or data field of eq. (1):
 *   DG_CONST     c[0]
 *   DG_AFFINE    c[0] + c[1] x + c[2] y
 *   DG_GAUSS_SUM sum_{i<m} c[4i+3] exp(-((x-c[4i])^2 + (y-c[4i+1])^2) / (2 c[4i+2]^2)),  m <= 4
 *   DG_QPOINTS   dev_vals: FP64 device values at the library's quadrature points
 *                (dg_mesh_qpoints): f uses the volume points, g^D / g^N the
 *                boundary-edge points.
 * eps, b and alpha must be DG_CONST or DG_AFFINE (DG_ERR_ARG otherwise).        */
typedef enum { DG_CONST = 0, DG_AFFINE = 1, DG_GAUSS_SUM = 2, DG_QPOINTS = 3 } dg_field_kind;

typedef struct {
    int32_t kind;
    int32_t m;
    double c[16];
    const double* dev_vals;
} dg_field;

/* Problem data of eq. (1) and the scheme parameters of eq. (ds).
 * kappa follows the method (SIPG -1, NIPG +1, IIPG 0, section 1).
 * sigma is the interior-edge penalty; sigma_D <= 0 selects 2*sigma on
 * Dirichlet edges (section 1: boundary penalty twice the interior one).
 * b0 is the superpenalty exponent of the penalty sigma eps / |e|^b0
 * (1 in the standard setting of the paper's set_parameter).               */
typedef struct {
    int32_t method;
    int32_t degree;
    double sigma;
    double sigma_D;
    double b0;
    dg_field eps, bx, by, alpha, f, gD, gN;
} dg_problem;

typedef struct {
    int64_t n_elems, n_int_edges, n_dir_edges, n_neu_edges;
    int64_t nnzb, n_dofs;
    int32_t degree, n_loc, n_q, n_qe; /* n_q = (k+2)^2 volume points, n_qe = k+2 points per edge */
    int32_t basis, reserved;          /* dg_basis of the mesh's tables */
    double h_max;                     /* largest edge length */
} dg_mesh_info;

typedef struct dg_mesh dg_mesh;
typedef struct dg_solver dg_solver;

/* Penalty and kappa of the paper's set_parameter (section 4): NIPG sigma = 1,
 * kappa = 1; SIPG sigma = 3k(k+1), kappa = -1; IIPG sigma = 3k(k+1), kappa = 0.
 * DG_ERR_METHOD for an unknown method, DG_ERR_DEGREE for k < 0 or
 * k > DG_MAX_DEGREE, or for SIPG / IIPG at k = 0 (sigma would be 0). */
int32_t dg_default_penalty(int32_t method, int32_t degree, double* sigma, double* kappa);

/* Builds the mesh from the arrays of section 2.1 (host, 0-based): nodes_xy
 * [n_nodes][2] FP64, elems [n_elems][3] counter-clockwise node ids,
 * dir_edges [n_dir][2] and neu_edges [n_neu][2] (start, end node; either
 * direction accepted).  Checks orientation, boundary classification and
 * manifoldness, builds edge connectivity, the BSR pattern and the reference
 * tables for `degree` in the Dubiner basis, and uploads them with
 * synchronous copies on the current device.  *out is NULL on error. */
int32_t dg_mesh_create(const double* nodes_xy, int64_t n_nodes, const int32_t* elems, int64_t n_elems,
                       const int32_t* dir_edges, int64_t n_dir, const int32_t* neu_edges, int64_t n_neu,
                       int32_t degree, dg_mesh** out);
/* dg_mesh_create with the element basis chosen (set_parameter's `base`,
 * section 4): DG_BASIS_DUBINER or DG_BASIS_MONOMIAL, else DG_ERR_ARG.  Every
 * call taking the mesh then works in that basis (coefficients, BSR blocks,
 * load vector); u_h itself does not depend on it.  With monomials the element
 * mass matrix is full (dg_euler_rhs applies it).  The batched calls
 * (dg_batch_*) build their own Dubiner meshes. */
int32_t dg_mesh_create_basis(const double* nodes_xy, int64_t n_nodes, const int32_t* elems, int64_t n_elems,
                             const int32_t* dir_edges, int64_t n_dir, const int32_t* neu_edges, int64_t n_neu,
                             int32_t degree, int32_t basis, dg_mesh** out);
int32_t dg_mesh_info_get(const dg_mesh* mesh, dg_mesh_info* out);
void dg_mesh_destroy(dg_mesh* mesh);

/* Uniform (red) refinement, the refinement step of the paper's driver
 * (section 2.1: the initial mesh is refined before assembly): every triangle
 * is split at its edge midpoints into four, and every listed boundary edge
 * into two halves of the same type.  dg_mesh_refine_sizes writes the refined
 * sizes (host int64[4]: n_nodes + n_edges, 4 n_elems, 2 n_dir_edges,
 * 2 n_neu_edges).  dg_mesh_refine writes the refined arrays in the layout of
 * dg_mesh_create into caller-owned device buffers of those sizes:
 * dev_nodes [.][2] FP64, dev_elems [.][3], dev_dir [.][2], dev_neu [.][2]
 * (int32, 0-based; dev_dir / dev_neu may be NULL when the list is empty).
 * Old nodes keep their index, the midpoint of an edge gets n_nodes + its edge
 * id (edges numbered in the order a walk over the elements and their edges
 * (v0 v1), (v1 v2), (v2 v0) first meets them); triangle K = (a, b, c) becomes
 * rows 4K..4K+3 = (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca);
 * boundary edge i = (a, b) becomes rows 2i, 2i+1 = (a, m), (m, b).
 * Stream-ordered, no synchronisation.  DG_ERR_ARG if an index of the refined
 * mesh would not fit int32. */
int32_t dg_mesh_refine_sizes(const dg_mesh* mesh, int64_t* sizes);
int32_t dg_mesh_refine(const dg_mesh* mesh, double* dev_nodes, int32_t* dev_elems, int32_t* dev_dir,
                       int32_t* dev_neu, void* stream);

/* Copies the BSR pattern into dev_row_ptr [n_elems+1] and dev_col_idx [nnzb]. */
int32_t dg_mesh_structure(const dg_mesh* mesh, int32_t* dev_row_ptr, int32_t* dev_col_idx, void* stream);

/* Coordinates of the quadrature points where DG_QPOINTS values are expected:
 * dev_vol_xy [n_elems][n_q][2]; dev_bnd_xy [n_bnd][n_qe][2] with n_bnd =
 * n_dir_edges + n_neu_edges; dev_bnd_normal [n_bnd][2] outward unit normals;
 * dev_bnd_type [n_bnd] (0 Dirichlet, 1 Neumann).  Any output may be NULL. */
int32_t dg_mesh_qpoints(const dg_mesh* mesh, double* dev_vol_xy, double* dev_bnd_xy, double* dev_bnd_normal,
                        int32_t* dev_bnd_type, void* stream);

/* L2 error of a DG solution (dg_error of section 2.4): ||u_h - u||_L2(Omega)
 * with a Stroud conical rule of q = k + 4 points per direction on every
 * element (exact for u_h^2), and h_max = the longest element edge.
 * dg_mesh_error_points writes that rule's physical points, dev_xy
 * [n_elems][(k+4)^2][2] (FP64, caller-owned), where the caller evaluates u.
 * dg_l2_error reads dev_x [n_dofs] (the coefficients) and dev_exact
 * [n_elems][(k+4)^2] (u at those points), writes *l2 and *h_max (host; either
 * may be NULL) and synchronises `stream`.  The sum is reduced in a fixed order
 * (deterministic) through a buffer owned by the mesh: calls on one mesh must
 * not overlap. */
int32_t dg_mesh_error_points(const dg_mesh* mesh, double* dev_xy, void* stream);
int32_t dg_l2_error(const dg_mesh* mesh, const double* dev_x, const double* dev_exact, double* l2, double* h_max,
                    void* stream);

/* Assembles the parts of D + C + R selected by `parts` into dev_vals
 * ([nnzb][n_loc][n_loc], FP64 if prec == DG_F64 else FP32) and the load
 * vector F_i = l_h(phi_i) (section 1 eq. (ds)) into dev_rhs ([n_dofs], same
 * precision), all in the given precision.  Every block has exactly one
 * writer, so the result is bitwise deterministic.  dev_rhs may be NULL.
 * problem->degree must equal the mesh degree. */
int32_t dg_assemble(const dg_mesh* mesh, const dg_problem* problem, int32_t prec, uint32_t parts,
                    void* dev_vals, void* dev_rhs, void* stream);

/* Restarted GMRES(restart) with right block-Jacobi preconditioning M =
 * blockdiag(A).  Stops when the true FP64 relative residual
 * ||F - A x||_2 / ||F||_2 <= rel_tol (checked after every Arnoldi cycle) or
 * after max_iters Arnoldi steps in total.  mixed = 1: the Arnoldi cycles run
 * in FP32 on an FP32 copy of A M^{-1} (iterative refinement: each cycle is an
 * inner solve of A d = r for the FP64 residual r, ended once its FP32 estimate
 * falls below inner_tol relative to ||r||, and x += d in FP64). */
typedef struct {
    int32_t restart;      /* Krylov dimension m per cycle, 1..4096 */
    int32_t max_iters;    /* cap on Arnoldi steps over all cycles */
    double rel_tol;       /* target relative residual (FP64, true residual) */
    int32_t mixed;        /* 0: FP64 cycles; 1: FP32 cycles + FP64 refinement */
    double inner_tol;     /* mixed only: per-cycle relative reduction target (e.g. 1e-5) */
    int32_t reorth;       /* 1: second classical Gram-Schmidt pass when the first loses > 1/sqrt(2) of the norm */
    int32_t profile;      /* 1: time the heavy kernels with HIP events on the solve stream (dg_solver_profile);
                             2: only the Gram-Schmidt dot kernel (two events per launch instead of ten per
                             block, for timing the solve with its dominant kernel); 3: as 2, and on the block
                             path each block's run of S SpMV launches under one pair of events (counted as S
                             launches, the gaps between them included); DG_ERR_ARG above 3 */
    double guess_limit;   /* the initial guess is replaced by zero when ||F - A x0|| > guess_limit ||F||
                             or is not finite; <= 0 selects 1 + 1e-8 (no worse than the zero guess;
                             the margin absorbs the rounding of the two norms); +inf keeps any finite guess */
    int32_t persistent;   /* one persistent workgroup runs the whole solve (one launch per solve, the same
                             algorithm) instead of one launch per GMRES kernel; it supports degree 1 or 2,
                             restart <= 512 and reorth = profile = 0.  0: automatic, taken for supported
                             systems of at most 4096 unknowns; 1: always (DG_ERR_ARG if unsupported);
                             -1: never */
    int32_t block;        /* Arnoldi vectors per Gram-Schmidt pass of the kernel-per-step path, S: 1 = one
                             (w = A M^{-1} v_j, then h = V^T w and w -= V h); S = 2, 3, 4, 6, 8, 16 or 32 = a
                             block of S vectors (w_0 from v_j, each next one from the one before, see basis)
                             projected on the basis in one pass, orthonormalised by Cholesky QR, its S
                             Hessenberg columns recovered from the block: the basis is read once per S
                             steps.  0 = automatic (with FP64 cycles 32 when restart <= 608, 16 when restart
                             <= 640; else 8, or 6 with mixed, when restart <= 2048; else 3; 1 with reorth).  A
                             block whose Gram matrix has an unresolvable pivot (Cholesky pivot <= 1e-8 of the
                             vector's norm) ends the cycle at the last column it determines.  With S >= 16 a
                             cycle that raises the true residual is undone (x restored), and it or a cycle ended
                             that way short of its length without converging halves S for the cycles after it.
                             S > 4 needs restart <= 2048, S = 16 restart <= 640 and S = 32 restart <= 608, both
                             with FP64 cycles (mixed = 0).  DG_ERR_ARG for other values, or for S > 1 with
                             reorth. */
    int32_t basis;        /* how a block's vectors are formed: 1 = monomial, w_i = A M^{-1} w_{i-1} (its Gram
                             matrix grows ill-conditioned with S: on the 256 x 256 P2 boundary-layer system
                             four vectors already take more steps); 2 = shifted by one,
                             w_i = (A M^{-1} - I) w_{i-1}, the products with the off-diagonal blocks of
                             A M^{-1} alone, which stay well conditioned (the same steps as one vector per
                             pass up to sixteen on the boundary-layer system); 0 = automatic (2).  The Krylov space is the same either way. */
} dg_solver_opts;

typedef struct {
    int32_t status;       /* DG_OK, DG_NOT_CONVERGED or an error */
    int32_t iters;        /* Arnoldi steps */
    int32_t cycles;       /* restart cycles (= refinement steps when mixed) */
    int32_t reorth_passes; /* second Gram-Schmidt passes taken */
    double rel_res;       /* true FP64 relative residual of the returned x */
    double rel_res0;      /* true FP64 relative residual of the initial guess */
    int32_t guess_rejected; /* 1: the initial guess failed the guess_limit test of the options
                               and was replaced by the zero guess */
    int32_t persistent;   /* dg_solver_solve: 1 if one persistent workgroup ran the solve
                             (opts.persistent); batch reports: 0 */
} dg_solve_report;

/* Allocates the Krylov workspace for `mesh` (device memory, owned by the
 * solver): restart+1 basis vectors, A M^{-1} without its identity diagonal
 * blocks and the inverse diagonal blocks, in the cycle precision. */
int32_t dg_solver_create(const dg_mesh* mesh, const dg_solver_opts* opts, dg_solver** out);
/* Block-Jacobi setup: inverts every diagonal block of A (FP64, Gauss-Jordan
 * with partial pivoting) and forms A M^{-1} in the cycle precision.  The
 * solver keeps dev_vals64 (FP64 BSR values, caller-owned, must stay valid and
 * unchanged until the last dg_solver_solve) for the true residual. */
int32_t dg_solver_setup(dg_solver* solver, const double* dev_vals64, void* stream);
/* Solves A x = F.  dev_x holds the initial guess on entry (zero for the plain
 * method) and the solution on exit.  The true FP64 residual judges the guess:
 * one whose residual norm exceeds opts.guess_limit ||F|| (or is not finite)
 * is replaced by the zero guess before the first cycle (report->guess_rejected = 1).  Synchronises `stream` before returning
 * so that `report` is filled.  DG_NOT_CONVERGED if max_iters was reached;
 * DG_ERR_NONFINITE if a residual norm became NaN / Inf. */
int32_t dg_solver_solve(dg_solver* solver, const double* dev_rhs, double* dev_x, dg_solve_report* report,
                        void* stream);
void dg_solver_destroy(dg_solver* solver);
/* The right block-Jacobi preconditioner of the last dg_solver_setup, for
 * inspection: dev_dinv64 [n_elems][n_loc][n_loc] (FP64) receives the inverse
 * of every diagonal block of A (M = blockdiag(A), section 2.3 eq. (system)),
 * row-major; dev_ahat [nnzb - n_elems][n_loc][n_loc] receives A M^{-1}
 * without its identity diagonal blocks, block rows in order and the
 * neighbour blocks of a row in the BSR order (block (K, L) = A_KL M_L^{-1}),
 * in the cycle precision (FP64, or FP32 when opts.mixed).  Either may be
 * NULL.  Stream-ordered copies; DG_ERR_ARG before a successful setup. */
int32_t dg_solver_preconditioner(dg_solver* solver, double* dev_dinv64, void* dev_ahat, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * block-Jacobi setup and GMRES of dg_solver_setup + dg_solver_solve for a
 * system small enough for the one-workgroup solve (opts.persistent = 1), with
 * no solver object and no allocation, no synchronisation and no memset, so
 * the call can be captured in a graph.  Same kernels, same results (bitwise)
 * and the same report as that path, the report written to dev_report
 * (device memory, caller-owned) when the kernels have run.  The setup's
 * outputs (D^{-1} FP64, A M^{-1} and D^{-1} in the cycle precision) go to a
 * fixed 4 MiB device array of the library that each device it runs on holds
 * until the process ends; calls on one device share it, so calls that overlap
 * on one device (other streams, or threads) race.  DG_ERR_ARG (nothing
 * launched) for restart > 128, reorth or profile set, a system whose setup
 * does not fit 4 MiB (n_elems n_loc^2 (8 + 2 p) + (nnzb - n_elems) n_loc^2 p
 * bytes with p = 8, or 4 when mixed, plus alignment) or whose Krylov state
 * does not fit one workgroup's LDS.  The report's status is
 * DG_ERR_NONFINITE when a diagonal block is singular or not finite. */
int32_t dg_solve_small_noalloc(const dg_mesh* mesh, const dg_solver_opts* opts, const double* dev_vals64,
                               const double* dev_rhs, double* dev_x, dg_solve_report* dev_report, void* stream);

/* Per-kernel statistics gathered when opts.profile = 1: for each heavy kernel
 * of the solve (spmv_hat, multidot, update, residual64, combine), the number
 * of launches that did work, their summed duration between HIP events
 * recorded on the solve stream, and their algorithmic HBM bytes (each
 * operand read or written once).  Writes up to `max` entries into `out`
 * (host) and their number into *count; reset = 1 clears the totals. */
typedef struct {
    char name[32];
    int64_t launches;
    double ms;
    double bytes;
} dg_kernel_stats;
int32_t dg_solver_profile(dg_solver* solver, dg_kernel_stats* out, int32_t max, int32_t* count, int32_t reset);

/* ------------------------------------------------------------------------
 * Non-linear reaction (section 3): alpha u - eps Lap u + b . grad u + r(u) = f
 * with the discrete system (D + C + R) v + H(v) = F, H_i(v) = int r(u_h) phi_i
 * (eq. (nonlinsystem)), solved by Newton's method, eq. (newton):
 * J w = -Res, v <- v + w, Res = (D + C + R) v + H(v) - F, J = D + C + R + HJ(v).
 * r is a polynomial without constant term, r(u) = sum_{p=1..n} c[p-1] u^p
 * (r(0) = 0 as section 3 requires; the paper's example is r(u) = u^2).  The
 * integrals use the volume rule of the assembly.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;            /* number of terms, 0..8 */
    int32_t reserved;
    double c[8];          /* c[p-1]: coefficient of u^p */
} dg_reaction;

/* H(v) (dev_h [n_dofs]) and the diagonal blocks of its Jacobian HJ_ij =
 * int r'(u_h) phi_j phi_i (dev_hj [n_elems][n_loc][n_loc], row = test i; HJ
 * is element-local, so it has no other blocks) at the coefficients dev_x,
 * FP64.  Either output may be NULL. */
int32_t dg_reaction_terms(const dg_mesh* mesh, const dg_reaction* r, const double* dev_x, double* dev_h,
                          double* dev_hj, void* stream);

typedef struct {
    int32_t max_newton;   /* cap on Newton steps */
    int32_t reserved;
    double tol;           /* stop when ||Res||_2 / ||F||_2 <= tol (checked before every step) */
} dg_newton_opts;

typedef struct {
    int32_t status;       /* DG_OK, DG_NOT_CONVERGED or an error */
    int32_t newton_steps; /* linear systems solved */
    int64_t linear_iters; /* GMRES iterations over all steps */
    double rel_res;       /* ||Res|| / ||F|| of the returned v (FP64) */
} dg_newton_report;

/* Newton's method for the mesh's system: dev_vals64 = D + C + R (FP64 BSR from
 * dg_assemble, caller-owned), dev_rhs = F, dev_x the initial guess on entry
 * (zero in the paper) and the solution on exit.  Each step solves J w = -Res
 * with `solver` (created for this mesh; its options set the linear tolerance,
 * restart and precision) from the zero guess.  Allocates the Jacobian's values
 * and three vectors for the duration of the call; synchronises `stream`.  On
 * return the solver holds no matrix (dg_solver_solve returns DG_ERR_ARG until
 * the next dg_solver_setup). */
int32_t dg_newton_solve(const dg_mesh* mesh, const dg_reaction* r, const dg_newton_opts* opts, dg_solver* solver,
                        const double* dev_vals64, const double* dev_rhs, double* dev_x, dg_newton_report* report,
                        void* stream);

/* Backward Euler in time (section 3: the linear reaction coefficient alpha of
 * its model stands for 1/dt of a time discretisation).  dev_vals64 = D + C + R
 * assembled (FP64) with alpha = alpha_0 + inv_dt, dev_rhs = F, dev_x = u^0 on
 * entry and u^{n_steps} on exit.  Step n solves, from the start u^n,
 *   (D + C + R) u^{n+1} [+ H(u^{n+1})] = F + inv_dt M u^n,
 * M the mass matrix (|det J_K| times the identity on element K for the
 * orthonormal basis, |det J_K| times the reference Gram matrix for the
 * monomials): by dg_solver_setup once and dg_solver_solve per step when
 * r is NULL, else by dg_newton_solve with nopts per step.  Allocates one vector
 * for the duration of the call; synchronises `stream`.  Stops at the first
 * step that does not reach its tolerance (report->status, report->steps). */
typedef struct {
    int32_t status;       /* DG_OK or the first failing step's status */
    int32_t steps;        /* time steps completed */
    int64_t linear_iters; /* GMRES iterations over all steps */
    int64_t newton_steps; /* Newton steps over all steps (0 without r) */
    double rel_res;       /* relative residual of the last step's system */
} dg_euler_report;
int32_t dg_implicit_euler(const dg_mesh* mesh, const dg_reaction* r, const dg_newton_opts* nopts, dg_solver* solver,
                          const double* dev_vals64, const double* dev_rhs, double inv_dt, int32_t n_steps,
                          double* dev_x, dg_euler_report* report, void* stream);
/* The step's load vector alone: dev_out = dev_rhs + inv_dt M dev_u (stream-ordered;
 * dev_out must not overlap dev_u). */
int32_t dg_euler_rhs(const dg_mesh* mesh, const double* dev_rhs, const double* dev_u, double inv_dt, double* dev_out,
                     void* stream);

/* y = b - A x in FP64 with the BSR values of the mesh (dev_b may be NULL: y = -A x). */
int32_t dg_residual(const dg_mesh* mesh, const double* dev_vals64, const double* dev_b, const double* dev_x,
                    double* dev_y, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent instances (own mesh, degree 1 or 2,
 * coefficients and data) assembled and solved by one persistent kernel
 * launch.  Per instance, the mesh arrays are those of dg_mesh_create and the
 * problem as in dg_assemble with these restrictions: degree 1 or 2; eps, b,
 * alpha DG_CONST or DG_AFFINE; f DG_CONST, DG_AFFINE or DG_GAUSS_SUM; g^D and
 * g^N DG_CONST or DG_AFFINE (no DG_QPOINTS).  The solve is the restarted
 * block-Jacobi GMRES of dg_solver_solve (FP64 true residual before each
 * cycle, FP64 or FP32 cycles) with a per-instance restart length
 * clamp(restart_min + restart_per_side * sqrt(n_elems / 2), 1, restart_max)
 * (sqrt(n_elems / 2) is the side N of an N x N structured grid).
 * Every instance is assembled by one element-parallel launch.  Instances with
 * fewer than lockstep_min_dofs unknowns are then solved by one persistent
 * launch (one workgroup per instance at a time, a queue ordered by decreasing
 * cost); larger ones by the lockstep solver, in which every Arnoldi step is
 * one launch per kernel over all of them (chunks of instances under a memory
 * budget), so that instances whose cost differs by orders of magnitude share
 * the whole GPU.
 * ------------------------------------------------------------------------ */
typedef struct {
    const double* nodes_xy;
    int64_t n_nodes;
    const int32_t* elems;
    int64_t n_elems;
    const int32_t* dir_edges;
    int64_t n_dir;
    const int32_t* neu_edges;
    int64_t n_neu;
    dg_problem problem;
} dg_instance;

typedef struct {
    int32_t mixed;            /* 0: FP64 cycles; 1: FP32 cycles + FP64 refinement */
    int32_t max_iters;        /* per instance */
    double rel_tol;           /* per instance, true FP64 relative residual */
    double inner_tol;         /* mixed only: per-cycle relative reduction target */
    int32_t restart_min;      /* restart length policy, see above; restart_max <= 512 */
    int32_t restart_max;
    double restart_per_side;
    int32_t block_threads;    /* persistent solve: threads per workgroup, 256 or 512 (0 = 512) */
    int32_t slots;            /* persistent solve: workgroups = workspace slots (0 = number of compute units) */
    int64_t lockstep_min_dofs; /* instances with at least this many unknowns use the lockstep solver */
    double lockstep_mem_gb;   /* lockstep workspace budget per chunk of instances (<= 0: 64 GB) */
    double guess_limit;       /* per instance, as dg_solver_opts.guess_limit */
    int32_t lockstep_block;   /* lockstep solver: Arnoldi vectors per Gram-Schmidt pass, as dg_solver_opts.block
                                 (1, 2, 3, 6 or 8; 0 = automatic = 8; DG_ERR_ARG otherwise) */
    int32_t lockstep_eager;   /* lockstep solver: 0 (default) records each restart cycle of a chunk once as a HIP
                                 graph and replays it; 1 launches the cycle's kernels one by one (same results) */
    int32_t lockstep_basis;   /* lockstep solver: block vectors as dg_solver_opts.basis (1 monomial, 2 shifted by
                                 one, 0 = automatic = 2) */
    int32_t reserved;
} dg_batch_opts;

typedef struct dg_batch dg_batch;

/* Validates and preprocesses every instance on the host (several threads),
 * uploads the concatenated arrays, and allocates one workspace per slot sized
 * for the largest instance.  Instance errors return that instance's code. */
int32_t dg_batch_create(const dg_instance* instances, int32_t count, const dg_batch_opts* opts, dg_batch** out);
/* Offsets of every instance's dofs in the concatenated solution vector
 * (host int64 [count + 1]; the last entry is the total). */
int32_t dg_batch_offsets(const dg_batch* batch, int64_t* x_offsets);
/* Assembles and solves every instance: dev_x (FP64, concatenated) holds the
 * initial guesses on entry and the solutions on exit; dev_reports
 * ([count], device) receives one report per instance.  Without lockstep
 * instances it is stream-ordered with no host synchronisation (so it can be
 * captured in a HIP graph); the lockstep solver synchronises the stream once
 * per restart cycle, and only then, to read two counters (the cycle itself is
 * one HIP graph replay unless opts.lockstep_eager is set). */
int32_t dg_batch_run(dg_batch* batch, double* dev_x, dg_solve_report* dev_reports, void* stream);
/* Progress callback for the lockstep part, called on the host thread of
 * dg_batch_run after every restart cycle with the number of lockstep
 * instances finished and their total. */
typedef void (*dg_progress_fn)(void* user, int32_t finished, int32_t total);
int32_t dg_batch_set_progress(dg_batch* batch, dg_progress_fn fn, void* user);
/* Number of instances the running (or last) dg_batch_run has started, read
 * with a copy on a separate non-blocking stream while the launch runs. */
int32_t dg_batch_progress(dg_batch* batch, int32_t* started);
/* Instance `instance` of the last dg_batch_run, for inspection.
 * dg_batch_system copies its FP64 BSR values (dev_vals64 [nnzb][n_loc][n_loc],
 * the layout of dg_assemble on the instance's mesh) and load vector
 * (dev_rhs [n_dofs]); either may be NULL.  dg_batch_preconditioner writes its
 * block-Jacobi preconditioner in the layout of dg_solver_preconditioner
 * (dev_dinv64 FP64, dev_ahat in the cycle precision), recomputed from those
 * FP64 values by the same kernels as the path that solved it (the persistent
 * workgroup's setup, or the lockstep setup launch of its chunk, which also
 * rewrites the chunk's own copies with the same values).  Stream-ordered;
 * DG_ERR_ARG for an index out of range or before the first dg_batch_run. */
int32_t dg_batch_system(const dg_batch* batch, int32_t instance, double* dev_vals64, double* dev_rhs, void* stream);
int32_t dg_batch_preconditioner(dg_batch* batch, int32_t instance, double* dev_dinv64, void* dev_ahat, void* stream);
void dg_batch_destroy(dg_batch* batch);

/* ------------------------------------------------------------------------
 * Learned initial guess: a multilayer perceptron Z_l = H_{l-1} W_l^T + b_l,
 * H_l = silu(Z_l) (identity on the last layer), trained and evaluated by the
 * library's own kernels: BF16 weights and activations as product operands,
 * FP32 accumulation (MFMA), FP32 master weights and Adam moments.
 * Parameters are one flat FP32 vector: W_1 ([w1][w0] row-major), b_1, W_2,
 * b_2, ...  All dev_ arrays are FP32 row-major [batch][width].
 * ------------------------------------------------------------------------ */
typedef struct dg_mlp dg_mlp;
/* widths[0..n_widths-1]: input, hidden..., output; init_params: host FP32
 * flat vector (dg_mlp_num_params values) copied into the model. */
int32_t dg_mlp_create(const int32_t* widths, int32_t n_widths, int32_t max_batch, const float* init_params,
                      dg_mlp** out);
int64_t dg_mlp_num_params(const dg_mlp* mlp);
/* Y = MLP(X) for B <= max_batch rows; keeps the activations for backward. dev_y may be NULL. */
int32_t dg_mlp_forward(dg_mlp* mlp, const float* dev_x, int32_t B, float* dev_y, void* stream);
/* For the last forward batch: loss = mean (Y - T)^2 (device scalar) and dY = dloss/dY. */
int32_t dg_mlp_loss_mse(dg_mlp* mlp, const float* dev_target, int32_t B, float* dev_dy, float* dev_loss, void* stream);
/* Gradients of sum(dY * Y) w.r.t. all parameters for the last forward batch (overwritten, not accumulated). */
int32_t dg_mlp_backward(dg_mlp* mlp, const float* dev_dy, int32_t B, void* stream);
/* One Adam step (step number t >= 1) with the last gradients. */
int32_t dg_mlp_adam_step(dg_mlp* mlp, float lr, float beta1, float beta2, float eps, int32_t t, void* stream);
/* Copies the FP32 parameters and / or gradients (either may be NULL). */
int32_t dg_mlp_params(dg_mlp* mlp, float* dev_params, float* dev_grads, void* stream);
void dg_mlp_destroy(dg_mlp* mlp);

/* Initial guesses on `mesh` from values on an nc x nc grid of cells of the
 * unit square (dev_coarse [B][nc*nc] FP32, cell (i, j) at index j*nc + i):
 * mode 0 = injection (each element takes its cell's value as a constant),
 * mode 1 = continuous piecewise-bilinear interpolation of the cell-centre
 * values with zero on the boundary, taken at the element vertices as a P1
 * function.  dev_x [B][ldx] FP64 coefficients in the mesh's basis (the
 * functions of degree above 1 get zero).
 * Synchronises `stream`. */
int32_t dg_warmstart_prolong(const dg_mesh* mesh, const float* dev_coarse, int32_t B, int32_t nc, int32_t mode,
                             double* dev_x, int64_t ldx, void* stream);

const char* dg_status_str(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* DGDCR_H */
