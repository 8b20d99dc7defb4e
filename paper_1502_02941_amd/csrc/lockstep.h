// Internal: lockstep batched GMRES (lockstep.hip), used by the batch object.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_internal.h"

namespace dg {

struct LsInst {
    int64_t T, n;
    int64_t vs;                // column stride of the instance's Krylov basis: n rounded up to LS_VALIGN rows
    int32_t k, m;              // degree, restart length
    int32_t id, id_local;      // batch instance index, index within the lockstep chunk
    int32_t nchunks, neblk;    // row chunks, element blocks
    int64_t rp_off, ci_off, val_off, x_off;               // batch arrays
    int64_t dinv_off, ahat_off, v_off, part_off;          // chunk buffers
    int64_t red_off, red2_off, hc_off, h_off, H_off;
    int64_t Hr_off;            // raw Hessenberg columns of the Arnoldi blocks
};

constexpr int LS_SMAX = 8;  // most Arnoldi vectors per Gram-Schmidt pass
// basis columns start on whole 32-row pieces (256 bytes in FP64, 128 in FP32): the dot kernel's staged pieces
// then never straddle a cache line (with columns starting at c n they straddled nearly always)
constexpr int64_t LS_VALIGN = 32;
inline int64_t ls_vstride(int64_t n) { return (n + LS_VALIGN - 1) / LS_VALIGN * LS_VALIGN; }

struct LsState {
    int32_t active, stop, J, mcyc, its, cycles, status, pad;
    double bnorm, beta, cyctol, invh;
    int32_t jb, bstep;         // Arnoldi blocks: first column and host step of the last block taken
    double ci[LS_SMAX * LS_SMAX];  // its inverse Cholesky factor, row-major block x block: q_i = sum_l u_l ci[l][i]
};

struct LsArgs {
    int32_t count;
    const LsInst* inst;
    LsState* state;
    const int64_t* eblk;  // [count+1] element-block prefix
    const int64_t* rblk;  // [count+1] row-chunk prefix
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const double* A64;
    const double* rhs;
    double* x;
    double* r;
    void* w;
    void* w1;             // the second vector of an Arnoldi block
    void* w2;             // the third (blocks of 3 or more)
    void* wx[LS_SMAX - 3];  // the fourth to eighth (blocks of 6 or 8)
    void* V;
    void* Ahat;
    void* DinvP;
    double* Dinv64;
    double* part;
    double* red;
    double* red2;
    double* hcol;
    double* H;
    double* Hr;
    double* cs;
    double* sn;
    double* g;
    double* y;
    dg_solve_report* reports;
    int* counters;
    double rel_tol, inner_tol, guess_limit;
    int32_t max_iters, mixed;
    int32_t block;        // Arnoldi vectors per Gram-Schmidt pass: 1, 2, 3, 6 or 8
    double theta;         // block vectors w_i = (Ahat - theta I) w_{i-1}: 0 monomial, 1 shifted
};

// One restart cycle of a lockstep chunk recorded as a HIP graph: recorded on
// the first cycle that needs it and replayed for every later cycle while the
// caller's solution and report buffers stay the same (the kernels' arguments
// hold those pointers).  Capture runs on a stream of its own (default
// priority, non-blocking); the graph is launched on the caller's stream.
struct LsGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key_x = nullptr;
    const void* key_rep = nullptr;
};
void ls_graph_release(LsGraph& g);

// Solves every instance of a chunk.  The host reads two counters once per
// restart cycle and nothing in between: every cycle launches all
// ceil(max_m / block) Arnoldi blocks, and the kernels of an instance whose
// cycle has ended return at once (the heavy ones also when every cycle of the
// chunk has ended).  With `graph`, each cycle after the first check is one
// replay of the recorded cycle.
int ls_solve(const LsArgs& A, int64_t n_eblk, int64_t n_rblk, int max_m, int mixed, hipStream_t st,
             dg_progress_fn fn, void* user, int done_before, int total, LsGraph* graph);
int64_t ls_elem_blocks(int k, int64_t T);
int64_t ls_row_chunks(int64_t n);
int ls_init(const LsArgs& A, hipStream_t st);
// block-Jacobi setup of every instance of a chunk: Dinv64, Ahat and DinvP (cycle precision)
int ls_setup(const LsArgs& A, int64_t n_eblk, int mixed, hipStream_t st);

}  // namespace dg
