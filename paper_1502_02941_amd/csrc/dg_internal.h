// Internal definitions of the gfx950 DG library (not part of the public ABI).
#pragma once

// An initial guess is replaced by zero when ||F - A x0|| > limit ||F|| (or is
// not finite).  Default limit: no worse than zero, with a margin above 1 that
// absorbs the rounding of the two norms (summed in different orders), so the
// zero guess itself is never flagged.
constexpr double GUESS_LIMIT_DEFAULT = 1.0 + 1e-8;
inline double guess_limit_of(double requested) { return requested > 0.0 ? requested : GUESS_LIMIT_DEFAULT; }

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/dgdcr.h"

#define DG_HIP_CHECK(expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return DG_ERR_HIP;             \
    } while (0)

namespace dg {

// Reference-table layout for degree k (shared by host code that fills the
// tables and the kernels that read them).  All entries are on the reference
// triangle {xi, eta >= 0, xi + eta <= 1}:
//   volume rule (Stroud conical product, q = k+2 points per direction):
//     w[g], xi[g], eta[g], then phi / dphi/dxi / dphi/deta [g][n]
//   edge rule (Gauss-Legendre, k+2 points on [0,1]): t[g], w[g], then for the
//     three local edges l (vertex l -> vertex l+1): phi / dxi / deta [l][g][n]
struct TabLayout {
    int n, nq, nqe;
    int vw, vxi, veta, vphi, vdx, vde, et, ew, ephi, edx, ede, size;
    __host__ __device__ constexpr explicit TabLayout(int k)
        : n((k + 1) * (k + 2) / 2), nq((k + 2) * (k + 2)), nqe(k + 2),
          vw(0), vxi(nq), veta(2 * nq), vphi(3 * nq), vdx(3 * nq + nq * n), vde(3 * nq + 2 * nq * n),
          et(3 * nq + 3 * nq * n), ew(3 * nq + 3 * nq * n + nqe), ephi(3 * nq + 3 * nq * n + 2 * nqe),
          edx(3 * nq + 3 * nq * n + 2 * nqe + 3 * nqe * n), ede(3 * nq + 3 * nq * n + 2 * nqe + 6 * nqe * n),
          size(3 * nq + 3 * nq * n + 2 * nqe + 9 * nqe * n) {}
};

// Reference tensors of the constant-coefficient assembly.  Each is an n x n
// matrix of integrals over the reference triangle or one of its edges,
// stored trial-major: entry (test i, trial j) at [j * n + i], so that the
// lane of trial function j reads a contiguous column.  Derivatives are with
// respect to the reference coordinates (xi, eta); edge integrals use the
// edge parameter t in [0, 1] (weights sum to 1); psi denotes the basis traced
// on the neighbour's edge lp at the same physical point (parameter 1 - t).
struct TenLayout {
    // volume: SXX = d_xi phi_i d_xi phi_j, SXY = d_xi phi_i d_eta phi_j + d_eta phi_i d_xi phi_j,
    // SYY = d_eta phi_i d_eta phi_j, CX = phi_i d_xi phi_j, CY = phi_i d_eta phi_j, MASS = phi_i phi_j
    static constexpr int VOL = 0;
    // edge l of K, index ED + 5 l + t: E = phi_i phi_j, DX = phi_i d_xi phi_j, DY = phi_i d_eta phi_j,
    // TX = d_xi phi_i phi_j, TY = d_eta phi_i phi_j
    static constexpr int ED = 6;
    // edge l of K against edge lp of the neighbour, index EO + 5 (3 l + lp) + t: F = phi_i psi_j,
    // GX = phi_i d_xi psi_j, GY = phi_i d_eta psi_j, HX = d_xi phi_i psi_j, HY = d_eta phi_i psi_j
    static constexpr int EO = 21;
    // for affine b: VB + t: xi phi_i d_xi phi_j, eta phi_i d_xi phi_j, xi phi_i d_eta phi_j, eta phi_i d_eta phi_j;
    // E1 + l: t phi_i phi_j on edge l; F1 + 3 l + lp: t phi_i psi_j
    static constexpr int VB = 66, E1 = 70, F1 = 73;
    static constexpr int COUNT = 82;
};

// The set the constant-coefficient kernel stages, one per method (kappa = -1,
// 0, 1 at index kappa + 1): the volume tensors, per local edge E and
// Z = kappa T - D (X and Y; the two normal-derivative terms of the diagonal
// block share their coefficient up to kappa), then the neighbour tensors.
struct TenStage {
    static constexpr int VOL = 0, ED = 6, EO = 15, VB = 60, E1 = 64, F1 = 67, COUNT = 76;
    static constexpr int CONST_B = 60;  // staged prefix used when b is constant
};
std::vector<double> stage_tensors(int k, const std::vector<double>& ten, double kappa);

// Tensor sets of the matrix-core assembly (k = 2, 3): each tensor is one row
// of nnp = 16 ceil(n^2 / 16) values in block order (entry (test i, trial j)
// at i n + j, zero beyond n^2), so that the blocks of 16 elements are the
// product of their 16 x K coefficient rows with K such rows.
//   diagonal set, per kappa:  VOL 0..5 (SXX SXY SYY CX CY MASS), VB 0..3, two zero
//                             rows, then per edge l: E, kappa TX - DX, kappa TY - DY, E1
//   neighbour set (l, lp):    F, GX, GY, HX, HY, F1, two zero rows
//   upwind points (any kappa): per edge l and point g (rows padded to PTS):
//                             w-free products phi_i(l, t_g) phi_j(l, t_g), then per
//                             (l, lp) and g: phi_i(l, t_g) psi_j(lp, 1 - t_g)
struct MfmaSet {
    static constexpr int DIAG = 24, OFF = 8;
    static constexpr int COUNT = DIAG + 9 * OFF;  // rows per kappa
    static constexpr int PTS = 8;                 // point rows per edge (k + 2 <= PTS)
    static constexpr int PCOUNT = 3 * PTS + 9 * PTS;
    __host__ __device__ static constexpr int nnp(int k) { return ((k + 1) * (k + 2) / 2 * ((k + 1) * (k + 2) / 2) + 15) / 16 * 16; }
};

// Field as seen by the kernels (same meaning as dg_field).
struct FieldDev {
    int32_t kind;
    int32_t m;
    double c[16];
    const double* vals;
};

struct AsmArgs {
    const double* xy;        // [T][6]: element vertex coordinates (x1,y1,x2,y2,x3,y3)
    const double* mL;        // [T][6]: per local edge l with a neighbour L, G_L^T (|e| n) (G = J^{-T}); 0 on boundary edges
    const int32_t* nbr;      // [T][3]: neighbour across local edge l, or -(b+1) for boundary edge b
    const int32_t* nbr_edge; // [T]: bits 2l..2l+1 = neighbour's local edge index
    const int32_t* row_ptr;  // [T+1]
    const int32_t* bnd_type; // [n_bnd]: 0 Dirichlet, 1 Neumann
    const void* tab;         // reference tables in the assembly precision
    int64_t T;
    double sigma, sigma_D, kappa, b0;
    uint32_t parts;
    FieldDev eps, bx, by, alpha, f, gD, gN;
    void* vals;
    void* rhs;
};

}  // namespace dg

struct dg_mesh {
    int k, n, nq, nqe;
    int64_t T, n_nodes, n_int, n_dir, n_neu, n_bnd, nnzb;
    double hmax;
    int device;
    // host copies
    std::vector<double> xy6;
    std::vector<int32_t> nbr, nbr_edge, row_ptr, col_idx, bnd_el, bnd_loc, bnd_type;
    std::vector<int32_t> bnd_elems;  // elements with at least one boundary edge, ascending
    std::vector<double> tab64;
    int32_t basis = DG_BASIS_DUBINER;
    double phi0 = 0.0;  // value of the constant basis function (sqrt 2 or 1)
    // device copies (owned)
    double* d_xy = nullptr;
    int32_t* d_nbr = nullptr;
    int32_t* d_nbr_edge = nullptr;
    int32_t* d_ebits = nullptr;   // [T]: neighbour edges (bits 2l, 2l+1), neighbour on l (8 + l), Neumann l (12 + l)
    int32_t* d_row_ptr = nullptr;
    int32_t* d_col_idx = nullptr;
    int32_t* d_bnd_type = nullptr;
    int32_t* d_bnd_el = nullptr;
    int32_t* d_bnd_loc = nullptr;
    int32_t* d_bnd_elems = nullptr;
    double* d_tab64 = nullptr;
    float* d_tab32 = nullptr;
    double* d_gt = nullptr;     // [T][6] neighbour gradient maps on the edges (see AsmArgs::mL)
    double* d_ten64 = nullptr;  // [3][TenStage::COUNT] staged tensors per kappa (k <= 3): n columns (trial j) of
                                //   test values i, each column zero-padded to whole 16-byte words
    float* d_ten32 = nullptr;
    double* d_tm64 = nullptr;   // [3][MfmaSet::COUNT][nnp] matrix-core tensor sets per kappa (k = 2, 3)
    float* d_tm32 = nullptr;
    double* d_tp64 = nullptr;   // [MfmaSet::PCOUNT][nnp] upwind point products (k = 2, 3)
    float* d_tp32 = nullptr;
    mutable void* d_mfcoef = nullptr;  // [47][T] (FP64 room): per-element coefficients of the matrix-core
                                       //   assembly (k = 2, 3), allocated by its first use; dg_assemble calls
                                       //   on one mesh that overlap in time race on it
    double* d_p1map = nullptr;  // [3][3]: P1 coefficients from vertex values (k >= 1)
    double* d_mref = nullptr;   // [n][n] reference mass matrix (monomial basis only)
    double* d_etab = nullptr;   // error rule (q = k + 4): w[nqr], xi[nqr], eta[nqr], phi[nqr][n]
    double* d_epart = nullptr;  // [ERR_BLOCKS + 1] partial sums of dg_l2_error
    int nqr = 0;
    // uniform refinement (dg_mesh_refine): the caller's arrays and one id per edge
    int64_t n_edges = 0;
    double* d_nodes = nullptr;    // [n_nodes][2]
    int32_t* d_elems = nullptr;   // [T][3]
    int32_t* d_eid = nullptr;     // [T][3] edge id of local edge l = (v_l, v_l+1)
    int32_t* d_owner = nullptr;   // [T][3] 1 where (K, l) is the first half-edge of its edge
    int32_t* d_dir = nullptr;     // [n_dir][2] as given
    int32_t* d_neu = nullptr;     // [n_neu][2] as given
    int32_t* d_dir_eid = nullptr;
    int32_t* d_neu_eid = nullptr;
};

namespace dg {
// Host-side reference tables for degree k (Golub-Welsch quadrature; the
// Dubiner basis in collapsed coordinates or the monomials, by dg_basis);
// returns TabLayout(k).size values.
std::vector<double> build_tables(int k, int basis);
void solver_invalidate(dg_solver* s);

// One-workgroup GMRES with its state in LDS (small.hip): byte offsets of each
// array in the dynamic LDS block.
struct SmallLayout {
    int64_t V, w0, w1, r, x, rp, ci, H, hcol, cs, sn, gv, yv, red, flag;
    int64_t ahat;   // A M^{-1} staged in LDS at this offset; -1: read from global memory
    int64_t bytes;
};
constexpr int SMALL_MAX_RESTART = 128;
struct SmallArgs {
    const double* A64;     // FP64 BSR values (true residual)
    const int32_t* rp;     // block row pointers [T + 1]
    const int32_t* ci;     // block column indices [nnzb]
    const void* Ahat;      // A D^{-1} without its diagonal blocks, cycle precision
    const void* Dinv;      // D^{-1} blocks, cycle precision
    const double* b;
    double* x;             // initial guess in, solution out
    dg_solve_report* rep;  // host-mapped pinned memory, or device memory
    const int* bad;        // non-null: set by the block-Jacobi setup when a pivot failed (the solve then
                           // only reports DG_ERR_NONFINITE)
    int64_t T;
    int32_t nnzb, m, max_iters, mixed;
    double rel_tol, inner_tol, guess_limit;
    SmallLayout L;
};
SmallLayout small_layout(int64_t T, int N, int64_t nnzb, int m, size_t ps, bool stage_ahat);
int small_lds_limit();
int small_prepare(int N, int mixed, const SmallLayout& L);
int small_launch(int N, int mixed, const SmallArgs& a, hipStream_t st);
// Block-Jacobi setup kernels of the solver (krylov.hip) on caller buffers:
// dinv64 [T][N][N] FP64, ahat [nnzb - T][N][N] and dinvp [T][N][N] in the cycle
// precision; *bad is set to 1 (never cleared) when a pivot fails.
int launch_block_jacobi(int N, int mixed, const double* A64, const int32_t* rp, const int32_t* ci, int64_t T,
                        double* dinv64, void* ahat, void* dinvp, int* bad, hipStream_t st);
// Error rule of dg_l2_error: Stroud q = k + 4; [w, xi, eta, phi[nqr][n]].
std::vector<double> build_error_table(int k, int basis, int* nqr);
constexpr int ERR_BLOCKS = 1024;
// Reference tensors (TenLayout) of degree k from the tables of build_tables.
std::vector<double> build_tensors(int k, const std::vector<double>& tab);
// Gauss-Jacobi rule for the weight (1-x)^a (1+x)^b on [-1,1].
void gauss_jacobi_gw(int n, double a, double b, double* x, double* w);
int launch_assemble(const dg_mesh* m, const AsmArgs& a, int prec, hipStream_t s);
int build_host_mesh(const double* xy, int64_t n_nodes, const int32_t* elems, int64_t T, const int32_t* dir,
                    int64_t n_dir, const int32_t* neu, int64_t n_neu, int32_t degree, dg_mesh* m, bool with_tables);
}  // namespace dg
