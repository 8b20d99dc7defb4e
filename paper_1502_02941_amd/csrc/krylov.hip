// Block-Jacobi preconditioned restarted GMRES on gfx950.
//
// Right preconditioning with M = blockdiag(A): GMRES runs on the operator
// A M^{-1}, formed once at setup as Ahat = A D^{-1} (block (K,L) = A_KL
// D_L^{-1}); its diagonal blocks are the identity and are not stored, so one
// operator application reads only the neighbour blocks.  x = x0 + D^{-1} V y.
//
// Each restart cycle:
//   r = F - A x in FP64 with the caller's FP64 matrix (true residual; the
//   host reads ||r|| once per cycle, its only synchronisation),
//   V_0 = r / ||r|| in the cycle precision P (double, or float when mixed),
//   Arnoldi steps j = 0.. : w = Ahat V_j; classical Gram-Schmidt h = V^T w,
//   w -= V h (a second pass when the norm drops by more than 1/sqrt(2)); the
//   Hessenberg column, Givens rotations and the residual estimate are updated
//   on the device by one thread, which raises a stop flag once the estimate
//   reaches the cycle target; every later kernel of the cycle then returns at
//   once, so the host enqueues a whole cycle without waiting;
//   y = H^{-1} g (device), x += D^{-1} (V y) with x in FP64.
// Mixed precision: P = float for Ahat, D^{-1}, V and the operator; the FP64
// residual and update make each cycle one step of iterative refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "dg_internal.h"
#include "mfma.h"

namespace dg {

enum { C_J = 0, C_STOP = 1, C_REORTH = 2, C_NREORTH = 3, C_NCTRL = 16 };
enum { S_BNORM2 = 0, S_RNORM2 = 1, S_INVH = 2, S_WNORM2 = 3, S_HN = 4, S_CYCTOL = 5, S_BETA = 6,
       S_QB = 7, S_NSCAL = 7 + 32 * 32 + 1 };  // S_QB..: the inverse Cholesky factor of an Arnoldi block (row-major, S x S)

constexpr int BLK = 256;
constexpr int MD_TARGET_BLOCKS = 2048;   // multidot: column tiles x row splits aimed at this many blocks
constexpr int MD_MIN_ROWS = 2048;        // multidot: fewest rows per split

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// out[slot] = sum of partials[0..count) in fixed order (one block)
__global__ __launch_bounds__(1024) void reduce_sum_kernel(const double* __restrict__ partials, int count,
                                                          double* out, int slot, const int* ctrl, int j,
                                                          int only_if_reorth)
{
    if (ctrl && (ctrl[C_STOP] || ctrl[C_J] != j || (only_if_reorth && !ctrl[C_REORTH]))) return;
    __shared__ double sh[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 1024) acc += partials[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += sh[w];
        out[slot] = t;
    }
}

// ---------------------------------------------------------------------------
// FP64 residual y = b - A x (A = full BSR incl. diagonal blocks); lane per
// (element, row i).  Optionally accumulates ||y||^2 into scal[slot].
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(BLK) void residual64_kernel(const double* __restrict__ A, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const double* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int64_t T, double* partials)
{
    constexpr int EPW = 64 / N;
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e;
    double v = 0.0;
    if (e < EPW && el < T) {
        double s = b ? b[el * N + i] : 0.0;
        const int s0 = rp[el], s1 = rp[el + 1];
        for (int sl = s0; sl < s1; ++sl) {
            const double* blk = A + ((int64_t)sl * N + i) * N;
            const double* xv = x + (int64_t)ci[sl] * N;
#pragma unroll
            for (int c = 0; c < N; ++c) s -= blk[c] * xv[c];
        }
        y[el * N + i] = s;
        v = s * s;
    }
    if (!partials) return;
    const double bs = block_sum(v, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// ||v||^2 of an FP64 vector into scal[slot]
__global__ __launch_bounds__(BLK) void norm2_kernel(const double* __restrict__ v, int64_t n, double* partials)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) acc += v[t] * v[t];
    const double bs = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// ---------------------------------------------------------------------------
// Setup: Dinv64 = inverse of every diagonal block (Gauss-Jordan with partial
// pivoting, one thread per element, matrix in LDS); then Ahat (P) and Dinv (P).
// ---------------------------------------------------------------------------
template <int N>
constexpr int inv_tpb() { return N <= 6 ? 64 : (N <= 10 ? 32 : 16); }

template <int N>
__global__ __launch_bounds__(inv_tpb<N>()) void invert_diag_kernel(const double* __restrict__ A,
                                                                   const int32_t* __restrict__ rp, int64_t T,
                                                                   double* __restrict__ Dinv, int* bad)
{
    constexpr int TPB = inv_tpb<N>();
    __shared__ double S[TPB][N * N];
    __shared__ int piv[TPB][N];
    const int t = threadIdx.x;
    const int64_t el = (int64_t)blockIdx.x * TPB + t;
    if (el >= T) return;
    double* M = S[t];
    const double* D = A + (int64_t)rp[el] * N * N;
    for (int q = 0; q < N * N; ++q) M[q] = D[q];
    for (int c = 0; c < N; ++c) {
        int p = c;
        double best = fabs(M[c * N + c]);
        for (int r = c + 1; r < N; ++r)
            if (fabs(M[r * N + c]) > best) { best = fabs(M[r * N + c]); p = r; }
        piv[t][c] = p;
        if (best == 0.0 || !isfinite(best)) { atomicExch(bad, 1); return; }
        if (p != c)
            for (int q = 0; q < N; ++q) { double tmp = M[c * N + q]; M[c * N + q] = M[p * N + q]; M[p * N + q] = tmp; }
        const double inv = 1.0 / M[c * N + c];
        M[c * N + c] = 1.0;
        for (int q = 0; q < N; ++q) M[c * N + q] *= inv;
        for (int r = 0; r < N; ++r) {
            if (r == c) continue;
            const double f = M[r * N + c];
            M[r * N + c] = 0.0;
            for (int q = 0; q < N; ++q) M[r * N + q] -= f * M[c * N + q];
        }
    }
    for (int c = N - 1; c >= 0; --c) {  // undo the row interchanges as column interchanges
        const int p = piv[t][c];
        if (p != c)
            for (int r = 0; r < N; ++r) { double tmp = M[r * N + c]; M[r * N + c] = M[r * N + p]; M[r * N + p] = tmp; }
    }
    double* out = Dinv + el * N * N;
    for (int q = 0; q < N * N; ++q) out[q] = M[q];
}

// Ahat block (K,L) = A_KL * Dinv_L in precision P; lane per (compact block, row i).
// Also converts Dinv to P for the solution update.
template <int N, typename P>
__global__ __launch_bounds__(BLK) void form_ahat_kernel(const double* __restrict__ A, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const double* __restrict__ Dinv64, int64_t T,
                                                        P* __restrict__ Ahat, P* __restrict__ DinvP)
{
    constexpr int EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e;
    if (e >= EPW || el >= T) return;
    const int s0 = rp[el], s1 = rp[el + 1];
    const int64_t c0 = (int64_t)s0 - el;  // compact index of the first neighbour block of row el
    for (int sl = s0 + 1; sl < s1; ++sl) {
        const double* a = A + ((int64_t)sl * N + i) * N;
        const double* d = Dinv64 + (int64_t)ci[sl] * N * N;
        P* out = Ahat + ((c0 + (sl - s0 - 1)) * N + i) * N;
        double arow[N];
#pragma unroll
        for (int k = 0; k < N; ++k) arow[k] = a[k];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) s += arow[k] * d[k * N + c];
            out[c] = (P)s;
        }
    }
    const double* dd = Dinv64 + (el * N + i) * N;
    P* dp = DinvP + (el * N + i) * N;
#pragma unroll
    for (int c = 0; c < N; ++c) dp[c] = (P)dd[c];
}

// ---------------------------------------------------------------------------
// Arnoldi kernels (precision P for vectors, FP64 for reductions)
// ---------------------------------------------------------------------------
// w = v + sum_L Ahat_KL v_L ; lane per (element, row i).  The grid is a
// multiple of 8 workgroups and workgroup b takes element group
// (b mod 8) (grid / 8) + b / 8: the hardware deals consecutive workgroups to
// the eight XCDs in turn, so each XCD sweeps one contiguous eighth of the
// elements and finds the neighbour blocks of v that the rows next to its own
// fetched in its own L2 (element-ordered meshes keep neighbours close).
inline int spmv_grid(int grid_elem) { return (grid_elem + 7) / 8 * 8; }
template <int N, typename P>
__global__ __launch_bounds__(BLK) void spmv_hat_kernel(const P* __restrict__ Ahat, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const P* __restrict__ Vbase,
                                                       int64_t n, P* __restrict__ w, int64_t T,
                                                       const int* __restrict__ ctrl, const P* __restrict__ vin,
                                                       P cid)
{
    if (ctrl[C_STOP]) return;
    constexpr int EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t grp = (int64_t)(blockIdx.x & 7) * (gridDim.x / 8) + (blockIdx.x >> 3);
    const int64_t el = (grp * 4 + wave) * EPW + e;
    if (e >= EPW || el >= T) return;
    const P* v = vin ? vin : Vbase + (int64_t)ctrl[C_J] * n;  // vin: the block's second product
    const int s0 = rp[el], s1 = rp[el + 1];
    const int64_t c0 = (int64_t)s0 - el;
    P s = cid * v[el * N + i];  // cid = 1 - theta: the identity blocks of Ahat - theta I
    if constexpr (N <= 6) {
        // A triangle has at most three neighbours: the loads of all three are
        // issued before the first product (absent ones read block 0 and
        // element 0, always allocated, and are not added), the sums keep the
        // neighbour order.
        constexpr int NB = 3;
        const int nb = s1 - s0 - 1;
        P bl[NB][N], xx[NB][N];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const bool has = q < nb;
            const P* blk = Ahat + (has ? ((c0 + q) * N + i) * N : 0);
            const P* xv = v + (has ? (int64_t)ci[s0 + 1 + q] * N : 0);
#pragma unroll
            for (int c = 0; c < N; ++c) {
                bl[q][c] = blk[c];
                xx[q][c] = xv[c];
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (q < nb) {
#pragma unroll
                for (int c = 0; c < N; ++c) s += bl[q][c] * xx[q][c];
            }
        for (int sl = s0 + 1 + NB; sl < s1; ++sl) {  // not reached on triangle meshes
            const P* blk = Ahat + ((c0 + (sl - s0 - 1)) * N + i) * N;
            const P* xv = v + (int64_t)ci[sl] * N;
#pragma unroll
            for (int c = 0; c < N; ++c) s += blk[c] * xv[c];
        }
    } else {
        for (int sl = s0 + 1; sl < s1; ++sl) {
            const P* blk = Ahat + ((c0 + (sl - s0 - 1)) * N + i) * N;
            const P* xv = v + (int64_t)ci[sl] * N;
#pragma unroll
            for (int c = 0; c < N; ++c) s += blk[c] * xv[c];
        }
    }
    w[el * N + i] = s;
}

// h[c] = V_c . w for c = 0..j and ||w||^2 (column j+1): a tall-skinny GEMV.
// Block (tile, split) reduces CT columns over one row range, reading w once
// per tile, and writes one partial per (column, split); reduce_cols_kernel
// then sums the splits.  j is the host's iteration index; the kernels do
// nothing if the cycle has stopped or the device count differs.
constexpr int CT = 16;  // measured on 786432 unknowns: 8 and 16 equal, 32 10% slower
template <typename P>
__global__ __launch_bounds__(BLK) void multidot_kernel(const P* __restrict__ V, const P* __restrict__ w, int64_t n,
                                                       int j, int64_t rows_per_split, const int* ctrl,
                                                       double* __restrict__ partials, int only_if_reorth)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j || (only_if_reorth && !ctrl[C_REORTH])) return;
    __shared__ double sh[4][CT];
    const int ncols = j + 2;
    const int c0 = blockIdx.x * CT;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;
    const P* col[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) col[c] = (c0 + c <= j) ? V + (int64_t)(c0 + c) * n : w;  // c = j+1 -> w . w
    double acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BLK) {
        const double wv = (double)w[r];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] += (double)col[c][r] * wv;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) sh[wave][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < CT && c0 + (int)threadIdx.x < ncols) {
        const int c = threadIdx.x;
        partials[(int64_t)(c0 + c) * gridDim.y + blockIdx.y] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
    }
}

// hcol[c] = sum over the row splits of column c's partials; one wavefront per
// column, fixed summation order (deterministic).
__global__ __launch_bounds__(BLK) void reduce_cols_kernel(const double* __restrict__ partials, int ncols,
                                                          int splits, int j, const int* ctrl, double* hcol,
                                                          int only_if_reorth)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j || (only_if_reorth && !ctrl[C_REORTH])) return;
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
    if (c >= ncols) return;
    const double* pc = partials + (int64_t)c * splits;
    double acc = 0.0;
    for (int sp = lane; sp < splits; sp += 64) acc += pc[sp];
    acc = wave_sum(acc);
    if (lane == 0) hcol[c] = acc;
}

// The same sums for a block's projections R_v[c] (column v jc + c, v < S),
// written as R and, negated and transposed, as negRT[c S + v]: the operand
// layout of the matrix-core update (the coefficients of four consecutive basis
// columns for sixteen vectors are then 4 x 128 contiguous bytes).
__global__ __launch_bounds__(BLK) void reduce_cols_rt_kernel(const double* __restrict__ partials, int S, int jc,
                                                             int splits, int j, const int* ctrl, double* R,
                                                             double* negRT)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
    if (c >= S * jc) return;
    const double* pc = partials + (int64_t)c * splits;
    double acc = 0.0;
    for (int sp = lane; sp < splits; sp += 64) acc += pc[sp];
    acc = wave_sum(acc);
    if (lane == 0) {
        R[c] = acc;
        negRT[(int64_t)(c % jc) * S + c / jc] = -acc;
    }
}

// The Gram matrix of a block of 32 vectors from the matrix-core update's
// per-workgroup partials: GP_N values per split (three 16 x 16 products G00,
// G01, G11; value e = 256 p + 64 v + l is register v of lane l of product p),
// split-major.  Workgroup (cg, sg) sums splits sg per .. sg per + per - 1 of
// columns 64 cg .. 64 cg + 63, four waves in a fixed order; with G null it
// writes the sums to out[sg][e], else it expands them into the symmetric
// row-major 32 x 32 G (G01 also as G10).
constexpr int GP_N = 3 * 256;
__global__ __launch_bounds__(BLK) void reduce_gram_kernel(const double* __restrict__ parts, int nsplit, int per,
                                                          int j, const int* ctrl, double* __restrict__ out,
                                                          double* __restrict__ G)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    __shared__ double sh[BLK / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = (int)blockIdx.x * 64 + lane;
    const int s0 = (int)blockIdx.y * per, s1 = s0 + per < nsplit ? s0 + per : nsplit;
    double acc = 0.0;
    for (int sp = s0 + wave; sp < s1; sp += BLK / 64) acc += parts[(int64_t)sp * GP_N + e];
    sh[wave][lane] = acc;
    __syncthreads();
    if (wave) return;
    const double v = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
    if (!G) {
        out[(int64_t)blockIdx.y * GP_N + e] = v;
        return;
    }
    const int p = e >> 8, r = (e >> 6) & 3, l = e & 63;
    const int x = MfmaOp<double>::row(l >> 4, r), y = l & 15;  // D[x][y] of product p
    const int a = p == 2 ? 16 : 0, b = p == 0 ? 0 : 16;
    G[(a + x) * 32 + b + y] = v;
    if (p == 1) G[(b + y) * 32 + a + x] = v;
}

// w -= sum_{c<=j} h[c] V_c and ||w||^2 (into scal[S_WNORM2]); rows split over
// threads, columns unrolled by 4 to keep many loads in flight.  In the
// reorthogonalisation pass (reorth_pass != 0) it runs only when flagged.
constexpr int UPD_E = 4;
template <typename P>
__global__ __launch_bounds__(BLK) void update_kernel(const P* __restrict__ V, P* __restrict__ w, int64_t n, int j,
                                                     const int* ctrl, double* partials,
                                                     const double* __restrict__ hcol, int reorth_pass)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j || (reorth_pass && !ctrl[C_REORTH])) return;
    __shared__ double sh[4];
    const int64_t base = (int64_t)blockIdx.x * (BLK * UPD_E) + threadIdx.x;
    double wr[UPD_E];
    bool in[UPD_E];
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        in[e] = t < n;
        wr[e] = in[e] ? (double)w[t] : 0.0;
    }
    int c = 0;
    for (; c + 3 <= j; c += 4) {
        const double h0 = hcol[c], h1 = hcol[c + 1], h2 = hcol[c + 2], h3 = hcol[c + 3];
        const P* v0 = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e])
                wr[e] -= h0 * (double)v0[t] + h1 * (double)v0[t + n] + h2 * (double)v0[t + 2 * n] +
                         h3 * (double)v0[t + 3 * n];
        }
    }
    for (; c <= j; ++c) {
        const double h = hcol[c];
        const P* vc = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e]) wr[e] -= h * (double)vc[t];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        if (in[e]) {
            const P pv = (P)wr[e];
            w[base + (int64_t)e * BLK] = pv;
            acc += (double)pv * (double)pv;
        }
    }
    const double bs = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// One thread: reorthogonalisation decision (after the first pass) or the
// Hessenberg column, Givens rotations, residual estimate and stop flag.
__global__ void arnoldi_decide_kernel(int* ctrl, const double* hcol, double* scal, int want_reorth, int* rflags)
{
    if (ctrl[C_STOP]) return;
    const int j = ctrl[C_J];
    const double before = hcol[j + 1];  // ||w||^2 before the first pass
    ctrl[C_REORTH] = (want_reorth && scal[S_WNORM2] < 0.5 * before) ? 1 : 0;
    ctrl[C_NREORTH] += ctrl[C_REORTH];
    rflags[j] = ctrl[C_REORTH];
}

// Hessenberg column j, previous Givens rotations, new rotation, residual
// estimate and stop test.  One block of 64 threads stages the column and the
// rotations in LDS in chunks; thread 0 runs the sequential chain.
constexpr int GV_CHUNK = 1024;
constexpr int TS_MAXJ = 4096;  // largest restart
__global__ __launch_bounds__(64) void givens_kernel(int* ctrl, const double* __restrict__ hcol,
                                                    const double* __restrict__ hcol2, double* __restrict__ H,
                                                    double* __restrict__ cs, double* __restrict__ sn,
                                                    double* __restrict__ g, double* scal, int ldh, int mcyc)
{
    if (ctrl[C_STOP]) return;
    __shared__ double sc[GV_CHUNK], ss[GV_CHUNK], sh[GV_CHUNK + 1], so[GV_CHUNK];
    __shared__ double carry;
    const int j = ctrl[C_J];
    const bool re = ctrl[C_REORTH] != 0;
    double* col = H + (int64_t)j * ldh;  // column-major: H[i + j*ldh]
    if (threadIdx.x == 0) carry = hcol[0] + (re ? hcol2[0] : 0.0);
    __syncthreads();
    for (int i0 = 0; i0 < j; i0 += GV_CHUNK) {
        const int cnt = j - i0 < GV_CHUNK ? j - i0 : GV_CHUNK;
        for (int t = threadIdx.x; t < cnt; t += 64) {
            sc[t] = cs[i0 + t];
            ss[t] = sn[i0 + t];
            sh[t + 1] = hcol[i0 + t + 1] + (re ? hcol2[i0 + t + 1] : 0.0);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = carry;
            for (int t = 0; t < cnt; ++t) {
                const double b = sh[t + 1];
                so[t] = sc[t] * a + ss[t] * b;
                a = -ss[t] * a + sc[t] * b;
            }
            carry = a;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 64) col[i0 + t] = so[t];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double hn = sqrt(scal[S_WNORM2]);
    const double a = carry, b = hn;
    const double d = sqrt(a * a + b * b);
    cs[j] = d == 0.0 ? 1.0 : a / d;
    sn[j] = d == 0.0 ? 0.0 : b / d;
    col[j] = d;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    ctrl[C_J] = j + 1;
    ctrl[C_REORTH] = 0;
    scal[S_HN] = hn;
    const bool breakdown = !(hn > 1e-300) || !isfinite(hn);
    scal[S_INVH] = breakdown ? 0.0 : 1.0 / hn;
    if (fabs(g[j + 1]) <= scal[S_CYCTOL] || breakdown || j + 1 >= mcyc) ctrl[C_STOP] = 1;
}

// V_{j} = w * (1/h_{j,j-1}) (j already advanced by the Givens step)
template <typename P>
__global__ __launch_bounds__(BLK) void normalize_kernel(P* __restrict__ V, const P* __restrict__ w, int64_t n,
                                                        const int* ctrl, const double* scal)
{
    if (ctrl[C_STOP]) return;
    const P s = (P)scal[S_INVH];
    P* out = V + (int64_t)ctrl[C_J] * n;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) out[t] = w[t] * s;
}

// ---------------------------------------------------------------------------
// Arnoldi blocks of S = 2, 3 or 4 vectors.  From the last basis vector v_j a block
// forms w_0 = Ahat v_j and w_i = Ahat w_{i-1} (i < S), projects them against
// v_0..v_j with one pass over the basis (R = V^T W) and updates them with a
// second pass (U = W - V R, with the S x S Gram matrix U^T U), so the basis is
// read twice per S Arnoldi steps instead of twice per step.  With the upper
// Cholesky factor C of U^T U the new basis vectors are Q = U C^{-1}, and
// W = V R + Q C gives the Hessenberg columns: Ahat v_j = w_0 = V R_0 + c_00 q_0
// and, for i < S - 1, Ahat q_i = sum_{l<=i} (w_{l+1} - Ahat V R_l) (C^{-1})_{li}
// with Ahat V = V H.
// ---------------------------------------------------------------------------
constexpr int BS_MAX = 32;
// the block's vectors w_0..w_{S-1}, passed by value
template <typename P>
struct BlockVecs {
    P* w[BS_MAX];
};

// partial V_c . w_r (c = 0..j, r < S), stored at partials[(r (j+1) + c) splits + split].
// The basis is streamed with non-temporal loads, so the S vectors, which every
// column tile re-reads, stay in the caches (7% less time per launch at three
// vectors on 786432 unknowns).
// Tiles of md_block_ct(S) columns over about md_block_target(S) workgroups:
// measured on 786432 unknowns over a 538-step cycle, 8 columns and 4096
// workgroups took 14% less time than 16 and 2048 with two vectors, while
// with three 16 and 2048 took 12% less than 8 and 4096 (each block re-reads
// its S vectors once per tile), and four vectors were within 2% either way.
constexpr int md_block_ct(int S) { return S == 3 ? 16 : (S == 8 ? 6 : 8); }

// Sums NV per-lane values over the 64 lanes of a wave: while the count is even
// each exchange step keeps half of them (the half picked by the step's lane
// bit) and adds the partner's copy of that half, so the work halves per step;
// the rest are summed over the remaining lane bits.  On return lanes with
// (lane & full) == 0 hold the totals of values base .. base + n - 1 in a[0..n).
template <int NV>
__device__ __forceinline__ void wave_butterfly_sum(double (&a)[NV], int lane, int& base, int& n, int& full)
{
    base = 0;
    n = NV;
    full = 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        if (n % 2 == 0) {
            const int half = n / 2;
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int i = 0; i < NV / 2; ++i) {
                if (i < half) {
                    const double send = up ? a[i] : a[half + i];
                    const double recv = __shfl_xor(send, o);
                    a[i] = (up ? a[half + i] : a[i]) + recv;
                }
            }
            if (up) base += half;
            n = half;
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i)
                if (i < n) a[i] += __shfl_xor(a[i], o);
            full |= o;
        }
    }
}
constexpr int md_block_target(int S) { return S == 3 ? 2048 : 4096; }
template <typename P, int S>
__global__ __launch_bounds__(BLK) void multidot_block_kernel(const P* __restrict__ V, BlockVecs<P> W, int64_t n,
                                                             int j, int64_t rows_per_split, const int* ctrl,
                                                             double* __restrict__ partials)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    constexpr int CT2 = md_block_ct(S);
    __shared__ double sh[4][S * CT2];
    const P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = W.w[q];
    const int ncols = j + 1;
    const int c0 = blockIdx.x * CT2;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;
    const P* col[CT2];
#pragma unroll
    for (int c = 0; c < CT2; ++c) col[c] = (c0 + c < ncols) ? V + (int64_t)(c0 + c) * n : wv[0];  // past j: discarded
    double a[S][CT2];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
        for (int c = 0; c < CT2; ++c) a[q][c] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BLK) {
        double x[S];
#pragma unroll
        for (int q = 0; q < S; ++q) x[q] = (double)wv[q][r];
#pragma unroll
        for (int c = 0; c < CT2; ++c) {
            const double v = (double)__builtin_nontemporal_load(col[c] + r);
#pragma unroll
            for (int q = 0; q < S; ++q) a[q][c] += v * x[q];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (S * CT2 == 48 || S <= 2) {  // (with 32 or 64 values the exchanges' indexing spills to scratch)
        double flat[S * CT2];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int c = 0; c < CT2; ++c) flat[q * CT2 + c] = a[q][c];
        int base, nv, full;
        wave_butterfly_sum<S * CT2>(flat, lane, base, nv, full);
        if ((lane & full) == 0) {
#pragma unroll
            for (int k = 0; k < S * CT2; ++k)
                if (k < nv) sh[wave][base + k] = flat[k];
        }
    } else {
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int c = 0; c < CT2; ++c) {
                const double v = wave_sum(a[q][c]);
                if (lane == 0) sh[wave][q * CT2 + c] = v;
            }
    }
    __syncthreads();
    if (threadIdx.x < S * CT2) {
        const int rr = threadIdx.x / CT2, c = threadIdx.x - rr * CT2;
        if (c0 + c < ncols)
            partials[((int64_t)rr * ncols + c0 + c) * gridDim.y + blockIdx.y] =
                (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    }
}

// The same partials for blocks of eight vectors on the matrix cores: a
// workgroup takes MF_CT = 32 basis columns over its row range and forms
// R = V_tile^T W as FP64 16 x 16 x 4 products (two per step, one per 16
// columns; FP32 data converted; the eight vectors fill half of the 16 product
// columns), the sum over rows running inside the products instead of across
// lanes.  Each wave stages 32-row chunks of its columns and of the eight
// vectors in LDS with coalesced loads (a load instruction reads 32 consecutive
// rows of two vectors) and feeds the products from there, the next chunk's
// loads in flight meanwhile; the row stride of the staged chunks is padded so
// that the 16 lanes reading one row of 16 columns hit different banks.  Tiles
// of 32 columns re-read the block's vectors 8/32 as often as the basis, against
// 8/6 for the vector-ALU kernel.  Measured on 786432 unknowns over a 538-step
// cycle (per launch): 16 columns and 64-row chunks 359 us, 32 and 32 348 us,
// 48 and 32 353 us, 16 and 32 363 us; without the prefetch 364 us; 1024 or 4096
// workgroups instead of 2048 within 3%; four independent partial sums per
// product (so that no step waits for the previous one) no faster.
constexpr int MF_CT = 32, MF_CH = 32;  // basis columns per tile, rows per staged chunk
constexpr int mf_target_blocks() { return 2048; }
// basis columns per tile and rows per staged chunk of the dot kernel for blocks of 32 vectors (the Gram pass
// of a block keeps MF_CT and MF_CH); on 786432 unknowns over a 538-step cycle, 16 columns took 540 us per launch
// against 478 and chunks of 16 rows (half the LDS, three waves per SIMD instead of two) 819 us
constexpr int MF_CT_WIDE = 32, MF_CH_WIDE = 32;
constexpr int mf_ct(int S) { return S > 16 ? MF_CT_WIDE : MF_CT; }
inline int mf_grid(int ntile, int nsplit) { return (ntile * nsplit + 7) / 8 * 8; }
// S = 8 or 16; with GRAM the columns are the block's vectors themselves (j + 1
// = S of them: the Gram matrix of a block of sixteen after its update).
//
// The grid is one-dimensional, 8 ceil(ntile nsplit / 8) workgroups: the
// hardware deals consecutive workgroups to the eight XCDs in turn, so
// workgroup b is given tile and split from 8-way contiguous ranges,
// (b mod 8) ceil(ntile nsplit / 8) + b / 8, tiles fastest.  The tiles of one
// row split then run on one XCD, close in time, and the block's vectors over
// those rows are fetched into that XCD's L2 once instead of once per tile
// (sixteen vectors on 786432 unknowns: HBM reads per launch 2.40 -> 1.79 GB,
// 1.01 x the algorithmic bytes, the time per launch unchanged at 364 us: the
// kernel is held by the latency of its load -> LDS -> product chain, the matrix
// cores 27% busy).  Operands loaded straight into the product registers
// instead (16-byte loads, the four lanes of a column reading 64 contiguous
// bytes, no LDS) took 639 us: each load instruction then touches 16 columns.
template <typename P, int S = 8, bool GRAM = false>
__global__ __launch_bounds__(BLK) void multidot_mfma_kernel(const P* __restrict__ V, BlockVecs<P> W, int64_t n, int j,
                                                            int64_t rows_per_split, int ntile, int nsplit,
                                                            const int* ctrl, double* __restrict__ partials)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    const int total = ntile * nsplit, per = (total + 7) / 8;
    const int logical = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (logical >= total) return;
    const int tile = logical % ntile, split = logical / ntile;
    static_assert(S == 8 || S == 16 || S == 32, "eight, sixteen or 32 vectors");
    constexpr int CT = GRAM ? MF_CT : mf_ct(S);       // columns of this tile
    constexpr int CH = GRAM || S <= 16 ? MF_CH : MF_CH_WIDE;  // rows per staged chunk
    constexpr int STR = sizeof(P) == 8 ? CH + 1 : CH + 2;  // padded row stride (elements)
    constexpr int WPB = BLK / 64, NA = CT / 16, NB = S > 16 ? S / 16 : 1;
    using Op = MfmaOp<double>;  // FP32 data too: the dots are summed in FP64, as by the vector-ALU kernel
    using VR = typename Op::V;
    // each wave's staged columns, then its staged block vectors; after the row loop the waves' partial sums
    __shared__ __align__(16) P stage[WPB][(CT + S) * STR];
    static_assert(sizeof(stage) >= sizeof(double) * WPB * CT * S, "room for the partial sums");
    const int ncols = GRAM ? S : j + 1;
    const int c0 = tile * CT;
    const int64_t r0 = (int64_t)split * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, i = lane & 15;
    P* mv = stage[wave];
    P* mw = stage[wave] + CT * STR;
    const P* wv[S];
#pragma unroll
    for (int v = 0; v < S; ++v) wv[v] = W.w[v];
    VR acc[NA][NB];
#pragma unroll
    for (int h = 0; h < NA; ++h)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[h][b] = VR{0, 0, 0, 0};
    constexpr int LPC = 64 / CH;  // columns whose rows one load instruction covers (2 for 32-row chunks)
    P x[CT / LPC], y[S / LPC];
    // a chunk's rows into registers (the next chunk's loads are in flight during this chunk's products):
    // lane l loads row l % CH of columns (l / CH) + LPC c
    const int lr = lane % CH, lc = lane / CH;
    auto pick = [&](int base) -> const P* {  // wv[base + lc], selected among constant indices
        const P* p = wv[base % S];
#pragma unroll
        for (int u = 1; u < LPC; ++u)
            if (lc == u) p = wv[(base + u) % S];
        return p;
    };
    auto load = [&](int64_t cb) {
        const int64_t r = cb + lr;
        const bool in = r < r1;
#pragma unroll
        for (int c = 0; c < CT / LPC; ++c) {  // columns past j read column j and are discarded
            const int cc = c0 + LPC * c + lc;
            if constexpr (GRAM) {  // columns LPC c .. LPC c + LPC - 1 are vectors of the block (none past S)
                if (LPC * c < S) {
                    const P* col = pick(LPC * c);
                    x[c] = in ? col[r] : P(0);
                } else {
                    x[c] = P(0);
                }
            } else
                x[c] = in ? __builtin_nontemporal_load(V + (int64_t)(cc < ncols ? cc : j) * n + r) : P(0);
        }
#pragma unroll
        for (int v = 0; v < S / LPC; ++v) {
            const P* yp = pick(LPC * v);
            y[v] = in ? yp[r] : P(0);
        }
    };
    int64_t cb = r0 + (int64_t)wave * CH;
    if (cb < r1) load(cb);
    for (; cb < r1; cb += (int64_t)WPB * CH) {
#pragma unroll
        for (int c = 0; c < CT / LPC; ++c) mv[(LPC * c + lc) * STR + lr] = x[c];
#pragma unroll
        for (int v = 0; v < S / LPC; ++v) mw[(LPC * v + lc) * STR + lr] = y[v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (cb + (int64_t)WPB * CH < r1) load(cb + (int64_t)WPB * CH);
#pragma unroll
        for (int t = 0; t < CH / 4; ++t) {
            double b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = (double)mw[((16 * nb + i) & (S - 1)) * STR + 4 * t + q];
#pragma unroll
            for (int h = 0; h < NA; ++h) {
                const double a = (double)mv[(16 * h + i) * STR + 4 * t + q];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[h][nb] = Op::mac(a, i < S ? b[nb] : 0.0, acc[h][nb]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // lane (i, q) holds the dots of column 16 h + row(q, v) with vector 16 nb + i (i < S)
    __syncthreads();
    double(*red)[CT * S] = reinterpret_cast<double(*)[CT * S]>(&stage[0][0]);
    if (i < S) {
#pragma unroll
        for (int h = 0; h < NA; ++h)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[wave][(16 * h + Op::row(q, v)) * S + 16 * nb + i] = (double)acc[h][nb][v];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < CT * S; t += BLK) {
        const int c = t / S, v = t - c * S;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < WPB; ++w) sum += red[w][t];
        if (c0 + c < ncols) partials[((int64_t)v * ncols + c0 + c) * nsplit + split] = sum;
    }
}

// w_r -= sum_{c<=j} R_r[c] V_c for r < S (R_r = R + r (j+1)) in the first
// nchunk workgroups (the basis streamed with non-temporal loads: 11% less time
// per launch at three vectors on 786432 unknowns, and the block's vectors are
// still cached for the next SpMV), with the Gram partials of the results, pair k = (p, q),
// p <= q in the order (0,0), (0,1), (1,1), (0,2), (1,2), (2,2), (0,3), ..., at
// partials[k * nchunk + block].  The workgroups after them take one row t <= j
// per wave of the Hessenberg products the block's columns need,
// HX[l][t] = sum_{c<j} Hrow[t][c] R_l[c] (l < S - 1; Hrow holds the raw
// Hessenberg matrix row-major, so a row is read coalesced); column j is not
// formed yet and is added by the block's Givens kernel.
template <typename P, int S>
__global__ __launch_bounds__(BLK) void update_block_kernel(const P* __restrict__ V, BlockVecs<P> W, int64_t n, int j,
                                                           const int* ctrl, double* partials,
                                                           const double* __restrict__ R, int nchunk,
                                                           const double* __restrict__ Hrow, int ldr,
                                                           double* __restrict__ HX, int ldx)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    constexpr int NG = S * (S + 1) / 2;
    if ((int)blockIdx.x >= nchunk) {
        const int lane = threadIdx.x & 63;
        const int t = ((int)blockIdx.x - nchunk) * (BLK / 64) + (threadIdx.x >> 6);
        if (t > j) return;
        const double* hr = Hrow + (int64_t)t * ldr;
        double acc[S - 1];
#pragma unroll
        for (int l = 0; l < S - 1; ++l) acc[l] = 0.0;
        for (int c = (t > 0 ? t - 1 : 0) + lane; c < j; c += 64) {
            const double h = hr[c];
#pragma unroll
            for (int l = 0; l < S - 1; ++l) acc[l] += h * R[l * (j + 1) + c];
        }
#pragma unroll
        for (int l = 0; l < S - 1; ++l) {
            const double v = wave_sum(acc[l]);
            if (lane == 0) HX[l * ldx + t] = v;
        }
        return;
    }
    __shared__ double sh[4];
    P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = W.w[q];
    const int64_t base = (int64_t)blockIdx.x * (BLK * UPD_E) + threadIdx.x;
    double u[S][UPD_E];
    bool in[UPD_E];
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        in[e] = t < n;
#pragma unroll
        for (int q = 0; q < S; ++q) u[q][e] = in[e] ? (double)wv[q][t] : 0.0;
    }
    int c = 0;
    for (; c + 3 <= j; c += 4) {
        double h[S][4];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int m = 0; m < 4; ++m) h[q][m] = R[q * (j + 1) + c + m];
        const P* v0 = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e]) {
                const double a0 = (double)__builtin_nontemporal_load(v0 + t),
                             a1 = (double)__builtin_nontemporal_load(v0 + t + n),
                             a2 = (double)__builtin_nontemporal_load(v0 + t + 2 * n),
                             a3 = (double)__builtin_nontemporal_load(v0 + t + 3 * n);
#pragma unroll
                for (int q = 0; q < S; ++q) u[q][e] -= h[q][0] * a0 + h[q][1] * a1 + h[q][2] * a2 + h[q][3] * a3;
            }
        }
    }
    for (; c <= j; ++c) {
        double h[S];
#pragma unroll
        for (int q = 0; q < S; ++q) h[q] = R[q * (j + 1) + c];
        const P* vc = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e]) {
                const double a0 = (double)__builtin_nontemporal_load(vc + t);
#pragma unroll
                for (int q = 0; q < S; ++q) u[q][e] -= h[q] * a0;
            }
        }
    }
    double gs[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) gs[k] = 0.0;
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        if (in[e]) {
            const int64_t t = base + (int64_t)e * BLK;
            double r[S];
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const P pv = (P)u[q][e];
                wv[q][t] = pv;
                r[q] = (double)pv;
            }
            int k = 0;
#pragma unroll
            for (int q = 0; q < S; ++q)
#pragma unroll
                for (int p = 0; p <= q; ++p) gs[k++] += r[p] * r[q];
        }
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const double bs = block_sum(gs[k], sh);
        if (threadIdx.x == 0) partials[k * nchunk + blockIdx.x] = bs;
    }
}

// w_r -= sum_{c<=j} R_r[c] V_c for the sixteen vectors of a block (FP64 or
// FP32 data; 32 vectors take the matrix-core update below: here, one row per
// thread, their 32 strided coefficient loads per basis column made the launch
// 1009 us against 466), upw_rows(S) rows per thread, without Gram partials
// (136 pair sums per row would not fit in registers: wide blocks form their
// Gram matrix afterwards with the matrix-core dot kernel on the updated
// vectors).  The coefficients R_r[c] are wave-uniform (scalar loads); the
// workgroups after the first nchunk take the Hessenberg products, as in
// update_block_kernel.
constexpr int upw_rows(int S) { return S <= 16 ? 2 : 1; }
template <typename P, int S>
__global__ __launch_bounds__(BLK) void update_wide_kernel(const P* __restrict__ V, BlockVecs<P> W, int64_t n, int j,
                                                          const int* ctrl, const double* __restrict__ R, int nchunk,
                                                          const double* __restrict__ Hrow, int ldr,
                                                          double* __restrict__ HX, int ldx)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    constexpr int E = upw_rows(S);
    if ((int)blockIdx.x >= nchunk) {
        const int lane = threadIdx.x & 63;
        const int t = ((int)blockIdx.x - nchunk) * (BLK / 64) + (threadIdx.x >> 6);
        if (t > j) return;
        const double* hr = Hrow + (int64_t)t * ldr;
        double acc[S - 1];
#pragma unroll
        for (int l = 0; l < S - 1; ++l) acc[l] = 0.0;
        for (int c = (t > 0 ? t - 1 : 0) + lane; c < j; c += 64) {
            const double h = hr[c];
#pragma unroll
            for (int l = 0; l < S - 1; ++l) acc[l] += h * R[l * (j + 1) + c];
        }
#pragma unroll
        for (int l = 0; l < S - 1; ++l) {
            const double v = wave_sum(acc[l]);
            if (lane == 0) HX[l * ldx + t] = v;
        }
        return;
    }
    const int64_t base = (int64_t)blockIdx.x * (BLK * E) + threadIdx.x;
    double u[S][E];
    bool in[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        in[e] = t < n;
#pragma unroll
        for (int q = 0; q < S; ++q) u[q][e] = in[e] ? (double)W.w[q][t] : 0.0;
    }
    for (int c = 0; c <= j; ++c) {
        const P* vc = V + (int64_t)c * n;
        double a[E];
#pragma unroll
        for (int e = 0; e < E; ++e) a[e] = in[e] ? (double)__builtin_nontemporal_load(vc + base + (int64_t)e * BLK) : 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const double h = R[q * (j + 1) + c];
#pragma unroll
            for (int e = 0; e < E; ++e) u[q][e] -= h * a[e];
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (in[e]) {
            const int64_t t = base + (int64_t)e * BLK;
#pragma unroll
            for (int q = 0; q < S; ++q) W.w[q][t] = (P)u[q][e];
        }
    }
}

// The same update on the matrix cores (FP64 cycles): W_tile -= V_tile R as
// 16 x 16 x 4 FP64 products, a wave owning UPM_RT x 16 rows and all S columns
// (S / 16 product column groups).  For each four basis columns, lane (i, q)
// loads V[c + q][row i of each row tile] (16 consecutive rows of a column per
// 16 lanes) as the A operand and -R_{16 g + i}[c + q] as the B operand (from
// the transposed copy negRT, 128 contiguous bytes per four lanes' column); the
// accumulators start from the block's vectors (D[i][j] in lane j + 16 g',
// register v, rows g' + 4 v) and are stored back there.  Columns past j give
// zero operands.  The workgroups after the first nchunk take the Hessenberg
// products, as in update_wide_kernel.  The updated tile also gives this
// workgroup's share of the block's Gram matrix U^T U: register v of lane
// (y, g) holds row g + 4 v of column y, which is both the A operand U^T[y][g]
// and the B operand U[g][y] of a product over those four rows, so G00, G01 and
// G11 are 16 x 16 x 4 products of the accumulators themselves; the four waves'
// sums go to gpart[blockIdx.x][GP_N] (reduce_gram_kernel).
constexpr int UPM_RT = 4, UPM_PD = 6;
// workgroups of the row tiles (each wave 16 UPM_RT rows), and the splits one
// workgroup of the first Gram reduction pass sums
inline int upm_grid(int64_t n) { return (int)(((n + 16 * UPM_RT - 1) / (16 * UPM_RT) + BLK / 64 - 1) / (BLK / 64)); }
constexpr int GP_PER = 64;
template <typename P, int S>
__global__ __launch_bounds__(BLK) void update_mfma_kernel(P* __restrict__ V_, BlockVecs<P> W, int64_t n, int j,
                                                          const int* ctrl, const double* __restrict__ R,
                                                          const double* __restrict__ negRT, int nchunk,
                                                          const double* __restrict__ Hrow, int ldr,
                                                          double* __restrict__ HX, int ldx,
                                                          double* __restrict__ gpart)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    static_assert(sizeof(P) == 8 && S == 32 && BLK == 256, "FP64 blocks of 32, four waves (the Gram partials)");
    if ((int)blockIdx.x >= nchunk) {
        const int lane = threadIdx.x & 63;
        const int t = ((int)blockIdx.x - nchunk) * (BLK / 64) + (threadIdx.x >> 6);
        if (t > j) return;
        const double* hr = Hrow + (int64_t)t * ldr;
        // 16 products at a time (all S - 1 at once set this kernel's register count for its main path too)
        for (int l0 = 0; l0 < S - 1; l0 += 16) {
            double acc[16];
#pragma unroll
            for (int l = 0; l < 16; ++l) acc[l] = 0.0;
            for (int c = (t > 0 ? t - 1 : 0) + lane; c < j; c += 64) {
                const double h = hr[c];
#pragma unroll
                for (int l = 0; l < 16; ++l)
                    if (l0 + l < S - 1) acc[l] += h * R[(l0 + l) * (j + 1) + c];
            }
#pragma unroll
            for (int l = 0; l < 16; ++l) {
                const double v = wave_sum(acc[l]);
                if (lane == 0 && l0 + l < S - 1) HX[(l0 + l) * ldx + t] = v;
            }
        }
        return;
    }
    using Op = MfmaOp<double>;
    using VR = typename Op::V;
    constexpr int NB = S / 16, RT = UPM_RT;
    const P* __restrict__ V = V_;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4;
    const int64_t r0 = ((int64_t)blockIdx.x * (BLK / 64) + wave) * (16 * RT);
    const bool live = r0 < n;  // a wave past the last row still takes part in the Gram sum (with zeros)
    // this lane's block vectors (16 nb + i), picked once: indexing the pointer array by the lane's column
    // kept all S pointers live in registers
    P* wl[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        P* pw = W.w[16 * nb];
#pragma unroll
        for (int u = 1; u < 16; ++u)
            if (i == u) pw = W.w[16 * nb + u];
        wl[nb] = pw;
    }
    VR acc[RT][NB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = r0 + 16 * rt + Op::row(q, v);
                acc[rt][nb][v] = r < n ? (double)wl[nb][r] : 0.0;
            }
    const int jc = live ? j + 1 : 0;
    // UPM_PD chunks of four columns in flight per wave (one was too few to cover the memory latency; 4: 452, 6:
    // 447, 8: 530 us per launch on the 256 x 256 P2 system, the last at one wave per SIMD)
    constexpr int PD = UPM_PD;
    double a[PD][RT], b[PD][NB];
    auto load = [&](int u, int c0) {
        const int c = c0 + q;
        const bool in = c < jc;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t r = r0 + 16 * rt + i;
            a[u][rt] = in && r < n ? (double)__builtin_nontemporal_load(V + (int64_t)c * n + r) : 0.0;
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[u][nb] = in ? negRT[(int64_t)c * S + 16 * nb + i] : 0.0;
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) load(u, 4 * u);
    for (int c0 = 0; c0 < jc; c0 += 4 * PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            double ca[RT], cb[NB];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) ca[rt] = a[u][rt];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) cb[nb] = b[u][nb];
            load(u, c0 + 4 * (u + PD));  // past column j: zeros, no memory read (a slot is never left stale)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[rt][nb] = Op::mac(ca[rt], cb[nb], acc[rt][nb]);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t r = r0 + 16 * rt + Op::row(q, v);
                if (r < n) wl[nb][r] = (P)acc[rt][nb][v];
            }
    VR g[3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int v = 0; v < 4; ++v) g[p][v] = 0.0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            g[0] = Op::mac(acc[rt][0][v], acc[rt][0][v], g[0]);
            g[1] = Op::mac(acc[rt][0][v], acc[rt][1][v], g[1]);
            g[2] = Op::mac(acc[rt][1][v], acc[rt][1][v], g[2]);
        }
    __shared__ double gs[BLK / 64][GP_N];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int v = 0; v < 4; ++v) gs[wave][256 * p + 64 * v + lane] = g[p][v];
    __syncthreads();
    double* gp = gpart + (int64_t)blockIdx.x * GP_N;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int e = 256 * p + (int)threadIdx.x;
        gp[e] = (gs[0][e] + gs[1][e]) + (gs[2][e] + gs[3][e]);
    }
}

// One workgroup: Gram reduction, Cholesky (pivot i is resolvable when c_ii >
// 1e-8 sqrt(G_ii), pivot 0 when c_00 > 1e-300), the block's Hessenberg
// columns (raw copies in the row-major Hr, leading dimension ldr; rotated in H, leading
// dimension ldh), the previous Givens rotations applied to them in turn, new
// rotations, residual estimates and stop tests.  A block with p < S
// resolvable pivots takes columns j..j+p and ends the cycle (the next vector
// lies in the span to working accuracy); (C^{-1}) goes to scal for the
// normalisation.
constexpr int BG_T = 1024;
// threads of the block Givens kernel for blocks of S vectors: 16 and 32 take 512 (the Hessenberg products then
// have 256 registers per lane instead of 128)
constexpr int bg_threads(int S) { return S >= 16 ? 512 : BG_T; }
// Rotations 0..count-1 (cs, sn) applied to columns 0..ncol-1 of colv, lane i
// of the first wave taking column i; each column is a chain of dependent
// steps, so the LDS loads of eight steps are issued together.
constexpr int BG_UNROLL = 8;
// longest cycle of the block path for blocks of S vectors (the S Hessenberg
// columns of a block live in LDS)
constexpr int bg_maxj(int S) { return S <= 4 ? TS_MAXJ : (S <= 8 ? 2048 : (S <= 16 ? 640 : 608)); }
template <int LD>
__device__ void bg_rotate_cols(double (*colv)[LD], int ncol, int count, const double* __restrict__ cs,
                               const double* __restrict__ sn, double* sc, double* ss)
{
    const int i = threadIdx.x;
    __syncthreads();
    double a = i < ncol ? colv[i][0] : 0.0;
    for (int i0 = 0; i0 < count; i0 += GV_CHUNK) {
        const int cnt = count - i0 < GV_CHUNK ? count - i0 : GV_CHUNK;
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += (int)blockDim.x) {
            sc[t] = cs[i0 + t];
            ss[t] = sn[i0 + t];
        }
        __syncthreads();
        if (i < ncol) {
            double* cv = colv[i] + i0;
            int t = 0;
            for (; t + BG_UNROLL <= cnt; t += BG_UNROLL) {
                double c[BG_UNROLL], s[BG_UNROLL], b[BG_UNROLL], o[BG_UNROLL];
#pragma unroll
                for (int u = 0; u < BG_UNROLL; ++u) {
                    c[u] = sc[t + u];
                    s[u] = ss[t + u];
                    b[u] = cv[t + u + 1];  // not yet written: this batch writes cv[t .. t + 7]
                }
#pragma unroll
                for (int u = 0; u < BG_UNROLL; ++u) {
                    o[u] = c[u] * a + s[u] * b[u];
                    a = -s[u] * a + c[u] * b[u];
                }
#pragma unroll
                for (int u = 0; u < BG_UNROLL; ++u) cv[t + u] = o[u];
            }
            for (; t < cnt; ++t) {
                const double b = cv[t + 1];
                cv[t] = sc[t] * a + ss[t] * b;
                a = -ss[t] * a + sc[t] * b;
            }
        }
    }
    if (i < ncol) colv[i][count] = a;
    __syncthreads();
}

template <int S>
__global__ __launch_bounds__(bg_threads(S)) void block_givens_kernel(int* ctrl, const double* __restrict__ gp, int nparts,
                                                            const double* __restrict__ R, double* __restrict__ Hr,
                                                            int ldr, const double* __restrict__ HX, int ldx,
                                                            double* __restrict__ H, int ldh,
                                                            double* __restrict__ cs, double* __restrict__ sn,
                                                            double* __restrict__ g, double* scal, int j, int mcyc,
                                                            double theta)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    constexpr int NT = bg_threads(S);
    constexpr int NG = S * (S + 1) / 2;
    // Hessenberg columns held in LDS at a time: a block of 32 forms and rotates its columns in two groups of 16
    // (32 columns of a 576-step cycle would not fit), keeping only their rows j.. for this block's rotations
    constexpr int GC = S < 16 ? S : 16, NGRP = S / GC, GS = S <= 8 ? S : 1;
    __shared__ double red[S <= 8 ? NG : 1][NT / 64];  // S >= 16: gp holds the reduced Gram matrix
    __shared__ double colv[GC][bg_maxj(S) + 4];
    __shared__ double h0s[NGRP > 1 ? bg_maxj(S) + 4 : 1];  // raw column j, when colv[0] is reused by a group
    __shared__ double sc[GV_CHUNK], ss[GV_CHUNK];
    __shared__ double G[GS][GS], Cf[S][S], Ci[S][S];  // in LDS: indexed dynamically
    __shared__ double tail[S][S + 2];  // rows j .. j + i + 1 of column j + i after the earlier rotations
    __shared__ int ncol_s, cut_s;
    double* h0 = NGRP > 1 ? h0s : colv[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (S <= 8) {
        double acc[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) acc[k] = 0.0;
        for (int t = threadIdx.x; t < nparts; t += NT)
#pragma unroll
            for (int k = 0; k < NG; ++k) acc[k] += gp[k * nparts + t];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) red[k][wave] = v;
        }
    }
    for (int i = threadIdx.x; i <= j; i += NT) h0[i] = R[i];
    if constexpr (S > 8) {
        // sixteen or more vectors: the Cholesky factor and its inverse on the lanes of wave 0 (thread 0 alone
        // spent most of this kernel's time on them): lane q holds column q of the Gram matrix, the pivots and the
        // rows of the factor are shared by shuffles, and lane q then solves C x = e_q for column q of C^{-1}
        __shared__ int pok_s;
        for (int k = threadIdx.x; k < S * S; k += NT) Cf[k / S][k % S] = Ci[k / S][k % S] = 0.0;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int q = threadIdx.x;
            double a[S];
#pragma unroll
            for (int i = 0; i < S; ++i) a[i] = q < S ? gp[i * S + q] : 0.0;  // G[i][q]
            const double sg = q < S ? sqrt(gp[q * S + q]) : 0.0;           // sqrt(G[q][q]) for the pivot test
            int pok = 0;
            bool alive = true;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const double d = __shfl(a[k], k, 64);  // the updated pivot G[k][k]
                const double sgk = __shfl(sg, k, 64);
                const double ckk = d > 0.0 ? sqrt(d) : 0.0;
                const bool ok = isfinite(ckk) && (k == 0 ? ckk > 1e-300 : ckk > 1e-8 * sgk);
                if (alive) {  // the same on every lane
                    if (q == k) Cf[k][k] = isfinite(ckk) ? ckk : 0.0;
                    if (!ok) {
                        alive = false;
                    } else {
                        const double rkq = q > k && q < S ? a[k] / ckk : 0.0;  // C[k][q]
                        if (q > k && q < S) Cf[k][q] = rkq;
                        // row k of C back from LDS, one broadcast read per entry (the wave's LDS accesses run
                        // in order; the fences keep the compiler from moving the reads above the writes)
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                        for (int i = k + 1; i < S; ++i) {
                            const double rki = Cf[k][i];  // C[k][i]
                            if (i <= q) a[i] -= rki * rkq;
                        }
                        ++pok;
                    }
                }
            }
            if (q == 0) pok_s = pok;
        }
        __syncthreads();
        if (threadIdx.x < pok_s) {  // C x = e_q on the resolvable leading triangle
            const int q = threadIdx.x;
            // back substitution by columns: once x_m is known its products join the sums of the rows above,
            // so each step waits for one division and one multiply-add (in registers: the wide-block kernels
            // have 256 per lane)
            double x[S], v[S];
#pragma unroll
            for (int i = 0; i < S; ++i) v[i] = 0.0;
#pragma unroll
            for (int m = S - 1; m >= 0; --m) {
                x[m] = m > q ? 0.0 : (m == q ? 1.0 / Cf[m][m] : -v[m] / Cf[m][m]);
                if (m <= q)
#pragma unroll
                    for (int i = 0; i < S; ++i)
                        if (i < m) v[i] += Cf[i][m] * x[m];
            }
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (i <= q) Ci[i][q] = x[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            h0[j] += theta;  // A v_j = w_0 + theta v_j
            const int pok = pok_s;
            int ncol = S < mcyc - j ? S : mcyc - j;
            if (pok < S && ncol > pok + 1) ncol = pok + 1;
            ncol_s = ncol;
            cut_s = pok < S ? 1 : 0;
            h0[j + 1] = Cf[0][0];
        }
        for (int k = threadIdx.x; k < S * S; k += NT) scal[S_QB + k] = Ci[k / S][k % S];
    } else {
        __syncthreads();
        if (threadIdx.x == 0) {
            h0[j] += theta;  // A v_j = w_0 + theta v_j
            int k = 0;
            for (int q = 0; q < S; ++q)
                for (int p = 0; p <= q; ++p) {
                    double v = 0.0;
                    for (int w = 0; w < NT / 64; ++w) v += red[k][w];
                    G[p][q] = G[q][p] = v;
                    ++k;
                }
            // upper Cholesky factor, stopping at the first pivot that is not resolvable
            int pok = 0;
            for (int p = 0; p < S; ++p)
                for (int q = 0; q < S; ++q) Cf[p][q] = Ci[p][q] = 0.0;
            for (int i = 0; i < S; ++i) {
                double d = G[i][i];
                for (int m = 0; m < i; ++m) d -= Cf[m][i] * Cf[m][i];
                const double cii = d > 0.0 ? sqrt(d) : 0.0;
                const bool ok = isfinite(cii) && (i == 0 ? cii > 1e-300 : cii > 1e-8 * sqrt(G[i][i]));
                Cf[i][i] = isfinite(cii) ? cii : 0.0;
                if (!ok) break;
                for (int q = i + 1; q < S; ++q) {
                    double v = G[i][q];
                    for (int m = 0; m < i; ++m) v -= Cf[m][i] * Cf[m][q];
                    Cf[i][q] = v / cii;
                }
                ++pok;
            }
            // inverse of the resolvable leading triangle
            for (int i = 0; i < pok; ++i) {
                Ci[i][i] = 1.0 / Cf[i][i];
                for (int q = i + 1; q < pok; ++q) {
                    double v = 0.0;
                    for (int m = i; m < q; ++m) v += Ci[i][m] * Cf[m][q];
                    Ci[i][q] = -v / Cf[q][q];
                }
            }
            int ncol = S < mcyc - j ? S : mcyc - j;
            if (pok < S && ncol > pok + 1) ncol = pok + 1;
            ncol_s = ncol;
            cut_s = pok < S ? 1 : 0;
            h0[j + 1] = Cf[0][0];
            for (int p = 0; p < S; ++p)
                for (int q = 0; q < S; ++q) scal[S_QB + p * S + q] = Ci[p][q];
        }
    }
    __syncthreads();
    const int ncol = ncol_s;
    for (int i = threadIdx.x; i <= j + 1; i += NT) Hr[(int64_t)i * ldr + j] = h0[i];
    // columns j .. j + ncol - 1 in groups of GC: column j is h0; columns j+1 .. from it and the earlier raw
    // columns; then the earlier blocks' rotations on all the group's columns at once; rows below j are final
    for (int g0 = 0; g0 < ncol; g0 += GC) {
        const int gn = ncol - g0 < GC ? ncol - g0 : GC;
        __syncthreads();
        if constexpr (NGRP > 1) {
            if (g0 == 0)
                for (int t = threadIdx.x; t <= j + 1; t += NT) colv[0][t] = h0[t];
        }
        const int i1 = g0 > 0 ? g0 : 1;  // first column of the group formed here
        if (i1 < g0 + gn) {
            // column i at row t is sum_{l<i} e_t[l] (C^{-1})_{l,i-1}, e_t[l] = (A u_l)[t] = w_{l+1} + theta w_l -
            // A V R_l in the basis [V, Q]: the rows times the upper triangle of C^{-1} as FP64 16 x 16 x 4
            // matrix-core products, a wave taking 16 rows at a time; lane (c, k) forms e of row c of the tile for
            // l = k (mod 4) only, and holds C^{-1}[4 s + k][16 ct + c] as its B operands throughout
            using Op = MfmaOp<double>;
            constexpr int NS = (S - 1 + 3) / 4, NCT = (S - 1 + 15) / 16;
            const int lane = threadIdx.x & 63, c = lane & 15, k = lane >> 4;
            double bop[NCT][NS];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int l = 4 * q + k, col = 16 * ct + c;
                    bop[ct][q] = l < S - 1 && col < S - 1 ? Ci[l][col] : 0.0;
                }
            const int nrows = j + g0 + gn + 1;  // rows 0 .. j + g0 + gn
            for (int tile = threadIdx.x >> 6; tile * 16 < nrows; tile += NT / 64) {
                const int t = tile * 16 + c;  // row c of the tile (A operand)
                // row t of [R; C] (the block's coefficients on V below row j + 1, the Cholesky factor above)
                auto rc = [&](int m) -> double {
                    return m >= ncol ? 0.0
                                     : (t <= j ? R[m * (j + 1) + t] : (t - j - 1 <= m ? Cf[t - j - 1][m] : 0.0));
                };
                const double h = t <= j + 1 ? h0[t] : 0.0;  // (Hr R_l)[t]: columns below j from HX, column j here
                double aop[NS];
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int l = 4 * q + k;
                    if (l < S - 1) {
                        const double hx =
                            t <= j + 1 ? (t <= j ? HX[l * ldx + t] : 0.0) + h * R[l * (j + 1) + j] : 0.0;
                        aop[q] = rc(l + 1) + theta * rc(l) - hx;
                    } else {
                        aop[q] = 0.0;
                    }
                }
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct) {
                    typename Op::V acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < NS; ++q) acc = Op::mac(aop[q], bop[ct][q], acc);
                    // D[r][c] in lane c + 16 g, register v, r = Op::row(g, v): column i = 16 ct + c + 1
                    const int i = 16 * ct + c + 1;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = tile * 16 + Op::row(k, v);
                        if (i >= i1 && i < g0 + gn && row <= j + i + 1) colv[i - g0][row] = acc[v];
                    }
                }
            }
            __syncthreads();
            for (int i = i1; i < g0 + gn; ++i)
                for (int t = threadIdx.x; t <= j + i + 1; t += NT) Hr[(int64_t)t * ldr + j + i] = colv[i - g0][t];
        }
        bg_rotate_cols(colv, gn, j, cs, sn, sc, ss);
        for (int i = 0; i < gn; ++i) {
            for (int t = threadIdx.x; t < j; t += NT) H[t + (int64_t)(j + g0 + i) * ldh] = colv[i][t];
            for (int r = threadIdx.x; r <= g0 + i + 1; r += NT) tail[g0 + i][r] = colv[i][j + r];
        }
    }
    // this block's own rotations, pipelined over the lanes of wave 0: lane i holds rows j .. j + i + 1 of column
    // j + i; at step t lane t's column has had rotations 0 .. t - 1 applied, so its rows t and t + 1 give
    // rotation t, which every later column then takes at once (a column of thread-0 loops through LDS was the
    // slowest part of this kernel); the estimate and the stop test follow each rotation, then the columns
    // taken are written out
    __syncthreads();
    if (threadIdx.x < 64) {
        const int i = threadIdx.x;
        double tr[S + 2];
#pragma unroll
        for (int r = 0; r < S + 2; ++r) tr[r] = i < ncol && r <= i + 1 ? tail[i < S ? i : 0][r] : 0.0;
        const double tol = scal[S_CYCTOL];
        double gcur = g[j];
        int taken = ncol, stop = 0;
#pragma unroll
        for (int t = 0; t < S; ++t) {
            if (t >= ncol || stop) break;  // the same on every lane
            const double a = __shfl(tr[t], t, 64), b = __shfl(tr[t + 1], t, 64);
            const double d = sqrt(a * a + b * b);
            const double c = d == 0.0 ? 1.0 : a / d, sr = d == 0.0 ? 0.0 : b / d;
            if (i == t) tr[t] = d;
            if (i > t) {
                const double x0 = tr[t], x1 = tr[t + 1];
                tr[t] = c * x0 + sr * x1;
                tr[t + 1] = -sr * x0 + c * x1;
            }
            const double gnext = -sr * gcur;
            if (i == 0) {
                cs[j + t] = c;
                sn[j + t] = sr;
                g[j + t] = c * gcur;
            }
            gcur = gnext;
            if (fabs(gnext) <= tol || j + t + 1 >= mcyc || (t == ncol - 1 && cut_s)) {
                taken = t + 1;
                stop = 1;
            }
        }
        if (i < taken)
#pragma unroll
            for (int r = 0; r < S; ++r)
                if (r <= i) H[j + r + (int64_t)(j + i) * ldh] = tr[r];
        if (i == 0) {
            g[j + taken] = gcur;
            ctrl[C_J] = j + taken;
            ctrl[C_REORTH] = 0;
            if (stop) ctrl[C_STOP] = 1;
        }
    }
}

// q_i = sum_{l<=i} u_l (C^{-1})_{li} into V_{j+1+i} for the columns the block
// took (ctrl[C_J] = j + t): i <= t - 2, and i = t - 1 unless the cycle stopped
template <typename P, int S>
__global__ __launch_bounds__(BLK) void normalize_block_kernel(P* __restrict__ V, BlockVecs<P> W, int64_t n, int j,
                                                              const int* ctrl, const double* scal)
{
    const int t = ctrl[C_J] - j;  // columns the block took (<= 0: the cycle had stopped before it)
    const int nq = ctrl[C_STOP] ? t - 1 : t;
    if (t < 1 || t > S || nq < 1) return;
    const P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = W.w[q];
    // C^{-1} in LDS (at S = 16 its 256 entries would not fit in registers)
    __shared__ double ci[S][S];
    for (int k = threadIdx.x; k < S * S; k += BLK) ci[k / S][k % S] = scal[S_QB + k];
    __syncthreads();
    P* out = V + (int64_t)(j + 1) * n;
    for (int64_t r = (int64_t)blockIdx.x * BLK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLK) {
        double u[S];
#pragma unroll
        for (int q = 0; q < S; ++q) u[q] = (double)wv[q][r];
        constexpr int NU = S <= 8 ? S : 1;  // sixteen outputs: a loop, with C^{-1} read from LDS
#pragma unroll NU
        for (int i = 0; i < S; ++i) {
            if (i < nq) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < S; ++l)
                    if (l <= i) v += u[l] * ci[l][i];
                out[(int64_t)i * n + r] = (P)v;
            }
        }
    }
}

// The same for blocks of 32 (FP64) on the matrix cores, as the transposed
// product Q_tile^T = (C^{-1})^T U_tile^T: a wave owns NRM_RT x 16 rows; lane
// (i, k) takes (C^{-1})_{c+k, 16 nb + i} (zero below the diagonal) as the A
// operand and u_{c+k} at row i of the tile (16 consecutive rows per 16 lanes,
// zero for vectors past the ones taken, so no stale value reaches a sum) as the
// B operand.  Column 16 nb + g + 4 v, row i of the result is register v of lane
// i + 16 g, so a store writes 16 consecutive rows of four columns.  (Read from
// LDS as wave-uniform operands, C^{-1} cost 528 LDS reads per row.)  The
// vectors are read non-temporally (their last use) and the new basis columns
// written non-temporally: measured, the following SpMV and dot kernels then
// run faster (plain loads took 84 instead of 68 us per launch).
constexpr int NRM_RT = 4;
static_assert(NRM_RT == UPM_RT, "launched on the grid of the matrix-core update (upm_grid)");
template <typename P, int S>
__global__ __launch_bounds__(BLK) void normalize_mfma_kernel(P* __restrict__ V, BlockVecs<P> W, int64_t n, int j,
                                                             const int* ctrl, const double* __restrict__ scal)
{
    static_assert(sizeof(P) == 8 && S == 32, "FP64 blocks of 32");
    const int t = ctrl[C_J] - j;
    const int nq = ctrl[C_STOP] ? t - 1 : t;
    if (t < 1 || t > S || nq < 1) return;
    using Op = MfmaOp<double>;
    using VR = typename Op::V;
    constexpr int RT = NRM_RT, NC = S / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, k = lane >> 4;
    const int64_t r0 = ((int64_t)blockIdx.x * (BLK / 64) + wave) * (16 * RT);
    if (r0 >= n) return;  // no barrier below
    double b[RT][NC];
#pragma unroll
    for (int c4 = 0; c4 < NC; ++c4) {
        const int c = 4 * c4 + k;
        const P* src = W.w[4 * c4];
#pragma unroll
        for (int u = 1; u < 4; ++u)
            if (k == u) src = W.w[4 * c4 + u];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t r = r0 + 16 * rt + i;
            b[rt][c4] = c < nq && r < n ? (double)__builtin_nontemporal_load(src + r) : 0.0;
        }
    }
    double a[2][NC];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int c4 = 0; c4 < NC; ++c4) {
            const int c = 4 * c4 + k, col = 16 * nb + i;
            a[nb][c4] = c <= col ? scal[S_QB + c * S + col] : 0.0;
        }
    P* out = V + (int64_t)(j + 1) * n;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r = r0 + 16 * rt + i;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            VR acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c4 = 0; c4 < (nb ? NC : NC / 2); ++c4) acc = Op::mac(a[nb][c4], b[rt][c4], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = 16 * nb + Op::row(k, v);
                if (col < nq && r < n) __builtin_nontemporal_store((P)acc[v], out + (int64_t)col * n + r);
            }
        }
    }
}

// start of a cycle: V_0 = r / beta, g = (beta, 0, ...), counters reset
template <typename P>
__global__ __launch_bounds__(BLK) void cycle_init_kernel(P* __restrict__ V, const double* __restrict__ r, int64_t n,
                                                         int* ctrl, double* scal, double* g, double cyc_rel,
                                                         double abs_tol)
{
    const double beta = sqrt(scal[S_RNORM2]);
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK)
        V[t] = (P)(r[t] * inv);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl[C_J] = 0;
        ctrl[C_STOP] = 0;
        ctrl[C_REORTH] = 0;
        g[0] = beta;
        scal[S_BETA] = beta;
        scal[S_CYCTOL] = fmax(cyc_rel * beta, abs_tol);
    }
}

// y = R^{-1} g(0:J) with R = H(0:J,0:J) upper triangular (column-major,
// leading dimension ldh), by 64-column panels from the bottom: one wave solves
// the panel's triangle from LDS, then the whole block updates the remaining
// right-hand side with the panel's columns.
constexpr int TS_PB = 48;
__global__ __launch_bounds__(1024) void trisolve_kernel(const int* ctrl, const double* __restrict__ H,
                                                        const double* __restrict__ g, double* __restrict__ y,
                                                        int ldh)
{
    __shared__ double rhs[TS_MAXJ];
    __shared__ double tri[TS_PB][TS_PB + 1];
    __shared__ double ys[TS_PB];
    const int J = ctrl[C_J];
    for (int k = threadIdx.x; k < J; k += blockDim.x) rhs[k] = g[k];
    __syncthreads();
    for (int c1 = J; c1 > 0; c1 -= TS_PB) {
        const int c0 = c1 - TS_PB > 0 ? c1 - TS_PB : 0;
        const int pb = c1 - c0;
        for (int q = threadIdx.x; q < pb * pb; q += blockDim.x) {
            const int r = q % pb, c = q / pb;  // R(c0 + r, c0 + c)
            tri[r][c] = H[(c0 + r) + (int64_t)(c0 + c) * ldh];
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            double v = lane < pb ? rhs[c0 + lane] : 0.0;
            for (int i = pb - 1; i >= 0; --i) {
                const double yi = __shfl(v, i, 64) / tri[i][i];
                if (lane == i) ys[i] = yi;
                if (lane < i) v -= tri[lane][i] * yi;
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < c0; k += blockDim.x) {
            double s = rhs[k];
            int c = 0;
            for (; c + 16 <= pb; c += 16) {  // sixteen loads in flight, summed in column order as below
                double hv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) hv[u] = H[k + (int64_t)(c0 + c + u) * ldh];
#pragma unroll
                for (int u = 0; u < 16; ++u) s -= hv[u] * ys[c + u];
            }
            for (; c < pb; ++c) s -= H[k + (int64_t)(c0 + c) * ldh] * ys[c];
            rhs[k] = s;
        }
        for (int c = threadIdx.x; c < pb; c += blockDim.x) y[c0 + c] = ys[c];
        __syncthreads();
    }
}

// u = V(:,0:J) y; rows split over threads, columns unrolled by 4
template <typename P>
__global__ __launch_bounds__(BLK) void combine_kernel(const P* __restrict__ V, int64_t n, const int* ctrl,
                                                      const double* __restrict__ y, P* __restrict__ u)
{
    const int J = ctrl[C_J];
    const int64_t base = (int64_t)blockIdx.x * (BLK * UPD_E) + threadIdx.x;
    double acc[UPD_E];
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) acc[e] = 0.0;
    int c = 0;
    for (; c + 4 <= J; c += 4) {
        const double y0 = y[c], y1 = y[c + 1], y2 = y[c + 2], y3 = y[c + 3];
        const P* v0 = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (t < n)
                acc[e] += y0 * (double)v0[t] + y1 * (double)v0[t + n] + y2 * (double)v0[t + 2 * n] +
                          y3 * (double)v0[t + 3 * n];
        }
    }
    for (; c < J; ++c) {
        const double yc = y[c];
        const P* vc = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (t < n) acc[e] += yc * (double)vc[t];
        }
    }
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        if (t < n) u[t] = (P)acc[e];
    }
}

// x += Dinv u (x FP64); lane per (element, row i)
template <int N, typename P>
__global__ __launch_bounds__(BLK) void dinv_update_kernel(const P* __restrict__ Dinv, const P* __restrict__ u,
                                                          double* __restrict__ x, int64_t T)
{
    constexpr int EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e;
    if (e >= EPW || el >= T) return;
    const P* d = Dinv + (el * N + i) * N;
    const P* uk = u + el * N;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) s += (double)d[c] * (double)uk[c];
    x[el * N + i] += s;
}

}  // namespace dg

using namespace dg;

struct dg_solver {
    const dg_mesh* m = nullptr;
    dg_solver_opts o{};
    int N = 0;
    int64_t T = 0, n = 0, n_off = 0;
    int mixed = 0;
    int grid_elem = 0, grid_chunk = 0, grid_vec = 0;
    const double* A64 = nullptr;
    void* Ahat = nullptr;   // [n_off][N][N] in P
    void* Dinv = nullptr;   // [T][N][N] in P
    double* Dinv64 = nullptr;
    void* V = nullptr;      // [(m+1)][n] in P
    void* w = nullptr;      // [n] in P
    void* u = nullptr;      // [n] in P
    void* w2 = nullptr;     // [n] in P: the third vector of blocks of 3 or more
    void* w3 = nullptr;     // [n] in P: the fourth vector of blocks of 4 or more
    void* wx[BS_MAX - 4] = {};  // [n] in P: vectors 5..32 of larger blocks
    double* G16 = nullptr;      // [S][S] Gram matrix of a block of S >= 16 vectors (wide blocks only)
    int64_t npartials = 0;      // doubles in partials
    double* r = nullptr;    // [n] FP64
    double* xprev = nullptr;  // [n] FP64: x before a cycle of 16 or more vectors per pass (restored if it lost)
    double* partials = nullptr;
    double* hcol = nullptr;
    double* hcol2 = nullptr;
    double* Rb = nullptr;   // [block][restart + 2]: an Arnoldi block's projections
    double* RbT = nullptr;  // [restart + 2][block]: the same negated, transposed (blocks of 32)
    double* Hr = nullptr;   // [restart + 2][restart + 1]: raw Hessenberg matrix of the block path, row-major
    double* HX = nullptr;   // [block - 1][restart + 2]: its products with a block's projections
    int block = 1;          // Arnoldi vectors per Gram-Schmidt pass (1, 2, 3, 4, 6 or 8)
    double theta = 0.0;     // block basis w_i = (A M^{-1} - theta I) w_{i-1}: 0 monomial, 1 shifted
    double* H = nullptr;
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;
    double* y = nullptr;
    double* scal = nullptr;
    int* ctrl = nullptr;
    int* bad = nullptr;
    int* rflags = nullptr;  // [restart]: 1 if iteration j took the second Gram-Schmidt pass
    int small = 0;                   // one workgroup with its state in LDS solves the whole system
    SmallLayout sl{};
    dg_solve_report* h_rep = nullptr;  // pinned host report written by that kernel
    int ready = 0;
    // built-in profiler (opts.profile): HIP events around the heavy kernels
    struct Rec { int cls; double bytes; int j; int pass; hipEvent_t e0, e1; int nl; };  // nl: launches timed
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<Rec> pending;
    int64_t pl[8] = {0};
    double pms[8] = {0}, pbytes[8] = {0};
    // multidot split for iteration j: (column tiles, row splits, rows per split)
    void md_shape(int j, int* tiles, int* splits, int64_t* rows) const;
    // the same for the Arnoldi block of S vectors starting at column j
    void md_shape2(int j, int S, int* tiles, int* splits, int64_t* rows) const;
    void md_shape_mf(int j, int* tiles, int* splits, int64_t* rows, int ct = dg::MF_CT) const;
};

void dg_solver::md_shape(int j, int* tiles, int* splits, int64_t* rows) const
{
    const int ncols = j + 2;
    const int nt = (ncols + dg::CT - 1) / dg::CT;
    const int64_t max_splits = std::max<int64_t>(1, n / dg::MD_MIN_ROWS);
    int64_t sp = (dg::MD_TARGET_BLOCKS + nt - 1) / nt;
    sp = std::max<int64_t>(1, std::min<int64_t>(sp, max_splits));
    int64_t r = (n + sp - 1) / sp;
    r = (r + dg::BLK - 1) / dg::BLK * dg::BLK;
    *tiles = nt;
    *splits = (int)((n + r - 1) / r);
    *rows = r;
}

void dg_solver::md_shape2(int j, int S, int* tiles, int* splits, int64_t* rows) const
{
    const int ct = dg::md_block_ct(S);
    const int nt = (j + 1 + ct - 1) / ct;
    const int64_t max_splits = std::max<int64_t>(1, n / dg::MD_MIN_ROWS);
    int64_t sp = (dg::md_block_target(S) + nt - 1) / nt;
    sp = std::max<int64_t>(1, std::min<int64_t>(sp, max_splits));
    int64_t r = (n + sp - 1) / sp;
    r = (r + dg::BLK - 1) / dg::BLK * dg::BLK;
    *tiles = nt;
    *splits = (int)((n + r - 1) / r);
    *rows = r;
}

void dg_solver::md_shape_mf(int j, int* tiles, int* splits, int64_t* rows, int ct) const
{
    const int nt = (j + 1 + ct - 1) / ct;
    const int64_t max_splits = std::max<int64_t>(1, n / dg::MD_MIN_ROWS);
    int64_t sp = (dg::mf_target_blocks() + nt - 1) / nt;
    sp = std::max<int64_t>(1, std::min<int64_t>(sp, max_splits));
    int64_t r = (n + sp - 1) / sp;
    r = (r + dg::BLK - 1) / dg::BLK * dg::BLK;
    *tiles = nt;
    *splits = (int)((n + r - 1) / r);
    *rows = r;
}

enum { PK_SPMV = 0, PK_MULTIDOT = 1, PK_UPDATE = 2, PK_RESIDUAL = 3, PK_COMBINE = 4, PK_N = 5 };
static const char* PK_NAMES[PK_N] = {"spmv_hat", "multidot", "update", "residual64", "combine"};

static hipEvent_t prof_event(dg_solver* s)
{
    if (s->evused == s->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->evpool.push_back(e);
    }
    return s->evpool[s->evused++];
}

// brackets one launch: returns true if recording (call prof_end after the launch)
static bool prof_begin(dg_solver* s, hipStream_t st, int cls, double bytes, int j, int pass, int nl = 1)
{
    if (!s->o.profile || (s->o.profile >= 2 && cls != PK_MULTIDOT && !(s->o.profile == 3 && cls == PK_SPMV)))
        return false;
    dg_solver::Rec r{cls, bytes, j, pass, prof_event(s), prof_event(s), nl};
    if (!r.e0 || !r.e1) return false;
    hipEventRecord(r.e0, st);
    s->pending.push_back(r);
    return true;
}

static void prof_end(dg_solver* s, hipStream_t st, bool on)
{
    if (on) hipEventRecord(s->pending.back().e1, st);
}

// after a synchronisation: accumulate the launches that did work (iteration
// j < J of the cycle, and for second passes only when the flag was raised)
static void prof_flush(dg_solver* s, int J, const int* rflags)
{
    for (const auto& r : s->pending) {
        const bool eff = r.j < 0 || (r.j < J && (r.pass == 0 || (rflags && rflags[r.j])));
        if (!eff) continue;
        double bytes = r.bytes;
        if (r.j == -2) bytes = ((double)J + 1.0) * (double)s->n * (s->mixed ? 4.0 : 8.0);  // combine: J columns + u
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
        s->pl[r.cls] += r.nl;
        s->pms[r.cls] += ms;
        s->pbytes[r.cls] += bytes;
    }
    s->pending.clear();
    s->evused = 0;
}

static void solver_free(dg_solver* s)
{
    for (auto e : s->evpool) hipEventDestroy(e);
    s->evpool.clear();
    hipFree(s->rflags);
    hipFree(s->Ahat); hipFree(s->Dinv); hipFree(s->Dinv64); hipFree(s->V); hipFree(s->w); hipFree(s->u);
    hipFree(s->r); hipFree(s->partials); hipFree(s->hcol); hipFree(s->hcol2); hipFree(s->H); hipFree(s->cs);
    hipFree(s->Rb); hipFree(s->RbT); hipFree(s->Hr); hipFree(s->HX); hipFree(s->w2); hipFree(s->w3);
    for (void* p : s->wx) hipFree(p);
    hipFree(s->G16);
    hipFree(s->xprev);
    hipFree(s->sn); hipFree(s->g); hipFree(s->y); hipFree(s->scal); hipFree(s->ctrl); hipFree(s->bad);
    if (s->h_rep) hipHostFree(s->h_rep);
    s->h_rep = nullptr;
}

extern "C" int32_t dg_solver_create(const dg_mesh* m, const dg_solver_opts* o, dg_solver** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (!m || !o) return DG_ERR_ARG;
    if (o->restart < 1 || o->restart > 4096 || o->max_iters < 0 || !(o->rel_tol > 0) || (o->mixed != 0 && o->mixed != 1))
        return DG_ERR_ARG;
    if (o->mixed && !(o->inner_tol > 0 && o->inner_tol < 1)) return DG_ERR_ARG;
    if (o->persistent < -1 || o->persistent > 1 || o->profile < 0 || o->profile > 3) return DG_ERR_ARG;
    const bool block_ok = o->block == 0 || (o->block >= 1 && o->block <= 4) || o->block == 6 || o->block == 8 ||
                          o->block == 16 || o->block == 32;
    // sixteen or 32 vectors in FP64 cycles only (in FP32 the block's sixteenth power loses too much: on a P3 IIPG
    // test 3582 steps against 1581 for one vector per pass)
    if (!block_ok || (o->block > 1 && o->reorth) || (o->block >= 16 && o->mixed)) return DG_ERR_ARG;
    if (o->basis < 0 || o->basis > 2 || (o->block > 4 && o->restart > bg_maxj(o->block))) return DG_ERR_ARG;
    dg_solver* s = new (std::nothrow) dg_solver();
    if (!s) return DG_ERR_OOM;
    s->m = m;
    s->o = *o;
    s->o.guess_limit = guess_limit_of(o->guess_limit);
    s->N = m->n;
    s->T = m->T;
    s->n = m->T * m->n;
    s->n_off = m->nnzb - m->T;
    s->mixed = o->mixed;
    // automatic: 32 (or, for restarts up to 640, sixteen) vectors per pass in FP64 cycles, else eight; in FP32
    // cycles the rounding of the block's vectors makes eight take up to a fifth more steps on hard systems (six:
    // a few percent)
    s->block = o->block != 0 ? o->block
                             : (o->reorth ? 1
                                          : (!o->mixed && o->restart <= bg_maxj(32)
                                                 ? 32
                                                 : (!o->mixed && o->restart <= bg_maxj(16)
                                                        ? 16
                                                        : (o->restart <= bg_maxj(8) ? (o->mixed ? 6 : 8) : 3))));
    s->theta = o->basis == 1 ? 0.0 : 1.0;
    const int EPW = 64 / s->N;
    s->grid_elem = (int)((s->T + 4 * EPW - 1) / (4 * EPW));
    s->grid_chunk = (int)((s->n + BLK * UPD_E - 1) / (BLK * UPD_E));
    s->grid_vec = (int)std::min<int64_t>((s->n + BLK - 1) / BLK, 2048);
    const size_t ps = s->mixed ? sizeof(float) : sizeof(double);
    const int mm = o->restart;
    const size_t NN = (size_t)s->N * s->N;
    int64_t maxgrid = std::max(std::max(s->grid_elem, s->grid_chunk), s->grid_vec);
    for (int j = 0; j < mm; ++j) {  // multidot partials: splits x (j+2) columns
        int nt, sp;
        int64_t rows;
        s->md_shape(j, &nt, &sp, &rows);
        maxgrid = std::max<int64_t>(maxgrid, (int64_t)sp * (j + 2));
        for (int S = 2; S <= 8; ++S) {  // the vector-ALU dot kernel's block sizes (and 8, an upper bound)
            s->md_shape2(j, S, &nt, &sp, &rows);
            maxgrid = std::max<int64_t>(maxgrid, (int64_t)sp * (j + 1) * S);
        }
        for (const int ct : {dg::MF_CT, dg::MF_CT_WIDE}) {  // eight or more vectors
            s->md_shape_mf(j, &nt, &sp, &rows, ct);
            maxgrid = std::max<int64_t>(maxgrid, (int64_t)sp * (j + 1) * BS_MAX);
        }
    }
    maxgrid = std::max<int64_t>(maxgrid, BS_MAX * (BS_MAX + 1) / 2 * (int64_t)s->grid_chunk);
    {  // the matrix-core update's Gram partials and the first reduction pass's sums
        const int64_t gm = dg::upm_grid(s->n);
        maxgrid = std::max<int64_t>(maxgrid, (gm + (gm + dg::GP_PER - 1) / dg::GP_PER) * dg::GP_N);
    }
    {  // the Gram matrix of a wide block: S x S columns in the shape of column count S (at most BS_MAX)
        int nt, sp;
        int64_t rows;
        s->md_shape_mf(BS_MAX - 1, &nt, &sp, &rows);
        maxgrid = std::max<int64_t>(maxgrid, (int64_t)BS_MAX * BS_MAX * sp);
    }
    bool ok = true;
    auto al = [&](void** p, size_t bytes) { if (ok && hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) { *p = nullptr; ok = false; } };
    al(&s->Ahat, ps * NN * std::max<int64_t>(s->n_off, 1));
    al(&s->Dinv, ps * NN * s->T);
    al((void**)&s->Dinv64, sizeof(double) * NN * s->T);
    al(&s->V, ps * (size_t)(mm + 1) * s->n);
    al(&s->w, ps * s->n);
    al(&s->u, ps * s->n);
    al((void**)&s->r, sizeof(double) * s->n);
    al((void**)&s->partials, sizeof(double) * (size_t)maxgrid);
    s->npartials = maxgrid;
    al((void**)&s->hcol, sizeof(double) * (mm + 2));
    al((void**)&s->hcol2, sizeof(double) * (mm + 2));
    if (s->block > 1) {
        al((void**)&s->Rb, sizeof(double) * s->block * (size_t)(mm + 2));
        if (s->block == 32) al((void**)&s->RbT, sizeof(double) * s->block * (size_t)(mm + 2));
        al((void**)&s->Hr, sizeof(double) * (size_t)(mm + 2) * (mm + 1));
        al((void**)&s->HX, sizeof(double) * (s->block - 1) * (size_t)(mm + 2));
    }
    if (s->block > 2) al(&s->w2, ps * s->n);
    if (s->block > 3) al(&s->w3, ps * s->n);
    for (int q = 4; q < s->block; ++q) al(&s->wx[q - 4], ps * s->n);
    if (s->block >= 16) al((void**)&s->G16, sizeof(double) * s->block * s->block);
    if (s->block >= 16) al((void**)&s->xprev, sizeof(double) * s->n);
    al((void**)&s->H, sizeof(double) * (size_t)(mm + 1) * mm);
    al((void**)&s->cs, sizeof(double) * mm);
    al((void**)&s->sn, sizeof(double) * mm);
    al((void**)&s->g, sizeof(double) * (mm + 1));
    al((void**)&s->y, sizeof(double) * mm);
    al((void**)&s->scal, sizeof(double) * S_NSCAL);
    al((void**)&s->ctrl, sizeof(int) * C_NCTRL);
    al((void**)&s->bad, sizeof(int));
    al((void**)&s->rflags, sizeof(int) * mm);
    if (!ok) { solver_free(s); delete s; return DG_ERR_OOM; }
    if (hipMemset(s->ctrl, 0, sizeof(int) * C_NCTRL) != hipSuccess) { solver_free(s); delete s; return DG_ERR_HIP; }
    // A system whose Krylov state fits one workgroup's LDS is solved by one
    // launch: the ~8 launches of every Arnoldi step would leave the chip idle.
    if (o->persistent != -1 && mm <= SMALL_MAX_RESTART && !o->reorth && !o->profile) {
        const int64_t lim = small_lds_limit();
        SmallLayout L = small_layout(s->T, s->N, m->nnzb, mm, ps, true);
        if (L.bytes > lim) L = small_layout(s->T, s->N, m->nnzb, mm, ps, false);
        if (L.bytes <= lim) {
            const int r = small_prepare(s->N, s->mixed, L);
            if (r != DG_OK) { solver_free(s); delete s; return r; }
            if (hipHostMalloc((void**)&s->h_rep, sizeof(dg_solve_report), hipHostMallocDefault) != hipSuccess) {
                s->h_rep = nullptr;
                solver_free(s);
                delete s;
                return DG_ERR_OOM;
            }
            s->small = 1;
            s->sl = L;
        }
    }
    if (o->persistent == 1 && !s->small) { solver_free(s); delete s; return DG_ERR_ARG; }
    *out = s;
    return DG_OK;
}

extern "C" void dg_solver_destroy(dg_solver* s)
{
    if (!s) return;
    solver_free(s);
    delete s;
}

static int setup_all(dg_solver* s, hipStream_t st)
{
    const dg_mesh* m = s->m;
    DG_HIP_CHECK(hipMemsetAsync(s->bad, 0, sizeof(int), st));
    const int r = launch_block_jacobi(s->N, s->mixed, s->A64, m->d_row_ptr, m->d_col_idx, s->T, s->Dinv64, s->Ahat,
                                      s->Dinv, s->bad, st);
    if (r != DG_OK) return r;
    int bad = 0;
    DG_HIP_CHECK(hipMemcpyAsync(&bad, s->bad, sizeof(int), hipMemcpyDeviceToHost, st));
    DG_HIP_CHECK(hipStreamSynchronize(st));
    return bad ? DG_ERR_NONFINITE : DG_OK;
}

namespace dg {
template <int N>
static int block_jacobi_n(int mixed, const double* A64, const int32_t* rp, const int32_t* ci, int64_t T,
                          double* dinv64, void* ahat, void* dinvp, int* bad, hipStream_t st)
{
    constexpr int TPB = inv_tpb<N>();
    const int EPW = 64 / N;
    const int grid = (int)((T + 4 * EPW - 1) / (4 * EPW));
    hipLaunchKernelGGL((invert_diag_kernel<N>), dim3((unsigned)((T + TPB - 1) / TPB)), dim3(TPB), 0, st, A64, rp, T,
                       dinv64, bad);
    if (mixed)
        hipLaunchKernelGGL((form_ahat_kernel<N, float>), dim3(grid), dim3(BLK), 0, st, A64, rp, ci, (const double*)dinv64,
                           T, (float*)ahat, (float*)dinvp);
    else
        hipLaunchKernelGGL((form_ahat_kernel<N, double>), dim3(grid), dim3(BLK), 0, st, A64, rp, ci,
                           (const double*)dinv64, T, (double*)ahat, (double*)dinvp);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

int launch_block_jacobi(int N, int mixed, const double* A64, const int32_t* rp, const int32_t* ci, int64_t T,
                        double* dinv64, void* ahat, void* dinvp, int* bad, hipStream_t st)
{
    switch (N) {
    case 1: return block_jacobi_n<1>(mixed, A64, rp, ci, T, dinv64, ahat, dinvp, bad, st);
    case 3: return block_jacobi_n<3>(mixed, A64, rp, ci, T, dinv64, ahat, dinvp, bad, st);
    case 6: return block_jacobi_n<6>(mixed, A64, rp, ci, T, dinv64, ahat, dinvp, bad, st);
    case 10: return block_jacobi_n<10>(mixed, A64, rp, ci, T, dinv64, ahat, dinvp, bad, st);
    case 15: return block_jacobi_n<15>(mixed, A64, rp, ci, T, dinv64, ahat, dinvp, bad, st);
    }
    return DG_ERR_DEGREE;
}
}  // namespace dg

extern "C" int32_t dg_solver_setup(dg_solver* s, const double* A64, void* stream)
{
    if (!s || !A64) return DG_ERR_ARG;
    s->A64 = A64;
    s->ready = 0;
    hipStream_t st = (hipStream_t)stream;
    const int r = setup_all(s, st);
    if (r == DG_OK) s->ready = 1;
    return r;
}

// One restart cycle on the block path: blocks of S Arnoldi vectors from
// columns 0, S, 2S, ... until a block's kernels record the stop.
template <int N, typename P, int S>
static void block_cycle(dg_solver* s, hipStream_t st, int mcyc, double spmv_bytes)
{
    const dg_mesh* m = s->m;
    const int mm = s->o.restart;
    const double ps = (double)sizeof(P), nb = (double)s->n;
    P* V = (P*)s->V;
    BlockVecs<P> W{};  // u is free until the cycle's combine
    {
        void* const first[4] = {s->w, s->u, s->w2, s->w3};
        for (int q = 0; q < BS_MAX; ++q) W.w[q] = (P*)(q < 4 ? first[q] : s->wx[q - 4]);
    }
    const P cid = (P)(1.0 - s->theta);
    P* const* wv = W.w;
    for (int j = 0; j < mcyc; j += S) {
        int nt, sp;
        int64_t rows;
        constexpr bool MF = S == 8 || S == 16 || S == 32;  // blocks of eight or more: the dots on the matrix cores
        if (MF) s->md_shape_mf(j, &nt, &sp, &rows, mf_ct(S));
        else s->md_shape2(j, S, &nt, &sp, &rows);
        const double md_bytes = (j + 1.0 + S) * nb * ps, up_bytes = (j + 1.0 + 2 * S) * nb * ps;
        if ((int64_t)S * (j + 1) * sp > s->npartials) {  // the partials of this shape do not fit (a sizing bug)
            fprintf(stderr, "dgdcr: block dot partials %lld exceed %lld\n", (long long)S * (j + 1) * sp,
                    (long long)s->npartials);
            abort();
        }
        // profile 3: one event pair around the block's S SpMV launches (S launches, gaps included)
        const bool spmv_group = s->o.profile == 3;
        const bool prg = spmv_group && prof_begin(s, st, PK_SPMV, spmv_bytes * S, j, 0, S);
        for (int q = 0; q < S; ++q) {
            const bool pr = !spmv_group && prof_begin(s, st, PK_SPMV, spmv_bytes, j, 0);
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(spmv_grid(s->grid_elem)), dim3(BLK), 0, st,
                               (const P*)s->Ahat, m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, wv[q], s->T,
                               s->ctrl, (const P*)(q ? wv[q - 1] : nullptr), cid);
            prof_end(s, st, pr);
        }
        prof_end(s, st, prg);
        bool pr = prof_begin(s, st, PK_MULTIDOT, md_bytes, j, 0);
        if constexpr (MF)
            hipLaunchKernelGGL((multidot_mfma_kernel<P, S>), dim3(mf_grid(nt, sp)), dim3(BLK), 0, st, (const P*)V, W,
                               s->n, j, rows, nt, sp, (const int*)s->ctrl, s->partials);
        else
            hipLaunchKernelGGL((multidot_block_kernel<P, S>), dim3(nt, sp), dim3(BLK), 0, st, (const P*)V, W, s->n, j,
                               rows, (const int*)s->ctrl, s->partials);
        prof_end(s, st, pr);
        if constexpr (S == 32)
            hipLaunchKernelGGL(reduce_cols_rt_kernel, dim3((S * (j + 1) + 3) / 4), dim3(BLK), 0, st,
                               (const double*)s->partials, S, j + 1, sp, j, (const int*)s->ctrl, s->Rb, s->RbT);
        else
            hipLaunchKernelGGL(reduce_cols_kernel, dim3((S * (j + 1) + 3) / 4), dim3(BLK), 0, st,
                               (const double*)s->partials, S * (j + 1), sp, j, (const int*)s->ctrl, s->Rb, 0);
        pr = prof_begin(s, st, PK_UPDATE, up_bytes, j, 0);
        const int hrows = (j + 1 + BLK / 64 - 1) / (BLK / 64);  // workgroups of the Hessenberg products
        const double* gram = s->partials;  // Gram partials (pairs x grid_chunk), or at S >= 16 the reduced matrix
        if constexpr (S == 32) {  // 32 vectors: the update on the matrix cores, the Gram matrix from its tiles
            const int gm = upm_grid(s->n), sg = (gm + GP_PER - 1) / GP_PER;
            hipLaunchKernelGGL((update_mfma_kernel<P, S>), dim3(gm + hrows), dim3(BLK), 0, st, V, W, s->n, j,
                               (const int*)s->ctrl, (const double*)s->Rb, (const double*)s->RbT, gm,
                               (const double*)s->Hr, mm + 1, s->HX, mm + 2, s->partials);
            prof_end(s, st, pr);
            double* stage = s->partials + (int64_t)gm * GP_N;
            hipLaunchKernelGGL(reduce_gram_kernel, dim3(GP_N / 64, sg), dim3(BLK), 0, st, (const double*)s->partials,
                               gm, GP_PER, j, (const int*)s->ctrl, stage, nullptr);
            hipLaunchKernelGGL(reduce_gram_kernel, dim3(GP_N / 64, 1), dim3(BLK), 0, st, (const double*)stage, sg, sg,
                               j, (const int*)s->ctrl, nullptr, s->G16);
            gram = s->G16;
        } else if constexpr (S == 16) {
            const int g16 = (int)((s->n + BLK * upw_rows(S) - 1) / (BLK * upw_rows(S)));
            hipLaunchKernelGGL((update_wide_kernel<P, S>), dim3(g16 + hrows), dim3(BLK), 0, st, (const P*)V, W, s->n,
                               j, (const int*)s->ctrl, (const double*)s->Rb, g16, (const double*)s->Hr, mm + 1, s->HX,
                               mm + 2);
            prof_end(s, st, pr);
            int gt, gs;
            int64_t grows;
            s->md_shape_mf(S - 1, &gt, &gs, &grows);
            if ((int64_t)S * S * gs > s->npartials) {
                fprintf(stderr, "dgdcr: block Gram partials exceed %lld\n", (long long)s->npartials);
                abort();
            }
            hipLaunchKernelGGL((multidot_mfma_kernel<P, S, true>), dim3(mf_grid(gt, gs)), dim3(BLK), 0, st, (const P*)V,
                               W, s->n, j, grows, gt, gs, (const int*)s->ctrl, s->partials);
            hipLaunchKernelGGL(reduce_cols_kernel, dim3((S * S + 3) / 4), dim3(BLK), 0, st, (const double*)s->partials,
                               S * S, gs, j, (const int*)s->ctrl, s->G16, 0);
            gram = s->G16;
        } else {
            hipLaunchKernelGGL((update_block_kernel<P, S>), dim3(s->grid_chunk + hrows), dim3(BLK), 0, st, (const P*)V,
                               W, s->n, j, (const int*)s->ctrl, s->partials, (const double*)s->Rb, s->grid_chunk,
                               (const double*)s->Hr, mm + 1, s->HX, mm + 2);
            prof_end(s, st, pr);
        }
        hipLaunchKernelGGL((block_givens_kernel<S>), dim3(1), dim3(bg_threads(S)), 0, st, s->ctrl, gram,
                           s->grid_chunk, (const double*)s->Rb, s->Hr, mm + 1, (const double*)s->HX, mm + 2, s->H,
                           mm + 1, s->cs, s->sn, s->g, s->scal, j, mcyc, s->theta);
        if constexpr (S == 32)
            hipLaunchKernelGGL((normalize_mfma_kernel<P, S>), dim3(upm_grid(s->n)), dim3(BLK), 0, st, V, W, s->n, j,
                               (const int*)s->ctrl, (const double*)s->scal);
        else
            hipLaunchKernelGGL((normalize_block_kernel<P, S>), dim3(s->grid_vec), dim3(BLK), 0, st, V, W, s->n, j,
                               (const int*)s->ctrl, (const double*)s->scal);
    }
}

template <int N, typename P>
static int solve_np(dg_solver* s, const double* b, double* x, dg_solve_report* rep, hipStream_t st)
{
    const dg_mesh* m = s->m;
    const int mm = s->o.restart;
    s->pending.clear();
    s->evused = 0;
    P* V = (P*)s->V;
    P* w = (P*)s->w;
    // ||b||
    hipLaunchKernelGGL(norm2_kernel, dim3(s->grid_vec), dim3(BLK), 0, st, b, s->n, s->partials);
    hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)s->partials, s->grid_vec, s->scal,
                       (int)S_BNORM2, (const int*)nullptr, 0, 0);
    DG_HIP_CHECK(hipGetLastError());
    double hs[S_NSCAL];
    int hc[C_NCTRL];
    DG_HIP_CHECK(hipMemcpyAsync(hs, s->scal, sizeof(hs), hipMemcpyDeviceToHost, st));
    DG_HIP_CHECK(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(hs[S_BNORM2]);
    if (!std::isfinite(bnorm)) return DG_ERR_NONFINITE;
    DG_HIP_CHECK(hipMemsetAsync(s->ctrl + C_NREORTH, 0, sizeof(int), st));
    rep->iters = 0;
    rep->cycles = 0;
    rep->rel_res0 = 0.0;
    rep->guess_rejected = 0;
    rep->persistent = 0;
    if (bnorm == 0.0) {
        DG_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * s->n, st));
        DG_HIP_CHECK(hipStreamSynchronize(st));
        rep->rel_res = 0.0;
        rep->status = DG_OK;
        return DG_OK;
    }
    const double abs_tol = s->o.rel_tol * bnorm;
    const double cyc_rel = s->mixed ? s->o.inner_tol : 0.0;
    int its = 0;
    int status = DG_NOT_CONVERGED;
    const double ps = (double)sizeof(P);
    const double nb = (double)s->n;
    const double idx_bytes = 4.0 * (double)(s->T + 1 + m->nnzb);
    std::vector<int> hflags(s->o.profile ? mm : 0);
    // Blocks of 16 or more vectors can lose orthogonality on hard non-normal systems (the Gram matrix of a long
    // shifted power basis): a cycle that raises the true residual is undone (x restored) and, like a cycle cut
    // short by an unresolvable pivot without converging, halves the block for the cycles after it.
    int cur_block = s->block;
    double rel_last = 0.0;
    int last_mcyc = 0;
    bool cycle_ran = false;
    for (;;) {
        bool pr = prof_begin(s, st, PK_RESIDUAL, (double)m->nnzb * N * N * 8.0 + 3.0 * nb * 8.0 + idx_bytes, -1, 0);
        hipLaunchKernelGGL((residual64_kernel<N>), dim3(s->grid_elem), dim3(BLK), 0, st, s->A64, m->d_row_ptr,
                           m->d_col_idx, b, x, s->r, s->T, s->partials);
        prof_end(s, st, pr);
        hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)s->partials, s->grid_elem,
                           s->scal, (int)S_RNORM2, (const int*)nullptr, 0, 0);
        DG_HIP_CHECK(hipGetLastError());
        DG_HIP_CHECK(hipMemcpyAsync(hs, s->scal, sizeof(hs), hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipMemcpyAsync(hc, s->ctrl, sizeof(hc), hipMemcpyDeviceToHost, st));
        if (s->o.profile && s->o.reorth)
            DG_HIP_CHECK(hipMemcpyAsync(hflags.data(), s->rflags, sizeof(int) * mm, hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipStreamSynchronize(st));
        if (s->o.profile) prof_flush(s, cycle_ran ? hc[C_J] : 0, s->o.reorth ? hflags.data() : nullptr);
        if (cycle_ran) its += hc[C_J];
        const double rel = std::sqrt(hs[S_RNORM2]) / bnorm;
        if (cycle_ran && cur_block >= 16) {
            if (!(rel <= rel_last)) {  // lost: back to x before the cycle, its residual recomputed
                DG_HIP_CHECK(hipMemcpyAsync(x, s->xprev, sizeof(double) * s->n, hipMemcpyDeviceToDevice, st));
                cur_block /= 2;
                cycle_ran = false;
                rep->iters = its;
                if (its >= s->o.max_iters) {
                    rep->rel_res = rel_last;
                    status = DG_NOT_CONVERGED;
                    break;
                }
                continue;
            }
            if (hc[C_J] < last_mcyc && !(rel <= s->o.rel_tol)) cur_block /= 2;
        }
        cycle_ran = false;
        if (rep->cycles == 0 && !rep->guess_rejected && !(rel <= s->o.guess_limit)) {
            // the guess is worse than zero: restart from x = 0
            DG_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * s->n, st));
            rep->guess_rejected = 1;
            rep->rel_res0 = rel;
            continue;
        }
        if (rep->cycles == 0 && !rep->guess_rejected) rep->rel_res0 = rel;
        rep->rel_res = rel;
        rep->iters = its;
        rep->reorth_passes = hc[C_NREORTH];
        if (!std::isfinite(rel)) { status = DG_ERR_NONFINITE; break; }
        if (rel <= s->o.rel_tol) { status = DG_OK; break; }
        if (its >= s->o.max_iters) { status = DG_NOT_CONVERGED; break; }
        const int mcyc = std::min(mm, s->o.max_iters - its);
        if (cur_block >= 16) {
            DG_HIP_CHECK(hipMemcpyAsync(s->xprev, x, sizeof(double) * s->n, hipMemcpyDeviceToDevice, st));
            rel_last = rel;
        }
        last_mcyc = mcyc;
        cycle_ran = true;
        hipLaunchKernelGGL((cycle_init_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, s->r, s->n, s->ctrl,
                           s->scal, s->g, cyc_rel, abs_tol);
        const double spmv_bytes = (double)s->n_off * N * N * ps + 2.0 * nb * ps + idx_bytes;
        if (cur_block == 2) block_cycle<N, P, 2>(s, st, mcyc, spmv_bytes);
        if (cur_block == 3) block_cycle<N, P, 3>(s, st, mcyc, spmv_bytes);
        if (cur_block == 4) block_cycle<N, P, 4>(s, st, mcyc, spmv_bytes);
        if (cur_block == 6) block_cycle<N, P, 6>(s, st, mcyc, spmv_bytes);
        if (cur_block == 8) block_cycle<N, P, 8>(s, st, mcyc, spmv_bytes);
        if (cur_block == 16) block_cycle<N, P, 16>(s, st, mcyc, spmv_bytes);
        if constexpr (sizeof(P) == 8)  // 32 vectors: FP64 cycles only
            if (cur_block == 32) block_cycle<N, P, 32>(s, st, mcyc, spmv_bytes);
        for (int j = 0; cur_block == 1 && j < mcyc; ++j) {
            int nt, sp;
            int64_t rows;
            s->md_shape(j, &nt, &sp, &rows);
            const double md_bytes = (j + 2.0) * nb * ps, up_bytes = (j + 3.0) * nb * ps;
            pr = prof_begin(s, st, PK_SPMV, spmv_bytes, j, 0);
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(spmv_grid(s->grid_elem)), dim3(BLK), 0, st,
                               (const P*)s->Ahat, m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, w, s->T, s->ctrl,
                               (const P*)nullptr, (P)1);
            prof_end(s, st, pr);
            pr = prof_begin(s, st, PK_MULTIDOT, md_bytes, j, 0);
            hipLaunchKernelGGL((multidot_kernel<P>), dim3(nt, sp), dim3(BLK), 0, st, (const P*)V, (const P*)w, s->n, j,
                               rows, (const int*)s->ctrl, s->partials, 0);
            prof_end(s, st, pr);
            hipLaunchKernelGGL(reduce_cols_kernel, dim3((j + 2 + 3) / 4), dim3(BLK), 0, st, (const double*)s->partials,
                               j + 2, sp, j, (const int*)s->ctrl, s->hcol, 0);
            pr = prof_begin(s, st, PK_UPDATE, up_bytes, j, 0);
            hipLaunchKernelGGL((update_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, w, s->n, j,
                               (const int*)s->ctrl, s->partials, s->hcol, 0);
            prof_end(s, st, pr);
            hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)s->partials, s->grid_chunk,
                               s->scal, (int)S_WNORM2, (const int*)s->ctrl, j, 0);
            if (s->o.reorth) {
                hipLaunchKernelGGL(arnoldi_decide_kernel, dim3(1), dim3(1), 0, st, s->ctrl, s->hcol, s->scal, 1,
                                   s->rflags);
                pr = prof_begin(s, st, PK_MULTIDOT, md_bytes, j, 1);
                hipLaunchKernelGGL((multidot_kernel<P>), dim3(nt, sp), dim3(BLK), 0, st, (const P*)V, (const P*)w,
                                   s->n, j, rows, (const int*)s->ctrl, s->partials, 1);
                prof_end(s, st, pr);
                hipLaunchKernelGGL(reduce_cols_kernel, dim3((j + 2 + 3) / 4), dim3(BLK), 0, st,
                                   (const double*)s->partials, j + 2, sp, j, (const int*)s->ctrl, s->hcol2, 1);
                pr = prof_begin(s, st, PK_UPDATE, up_bytes, j, 1);
                hipLaunchKernelGGL((update_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, w, s->n, j,
                                   (const int*)s->ctrl, s->partials, s->hcol2, 1);
                prof_end(s, st, pr);
                hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(1024), 0, st, (const double*)s->partials,
                                   s->grid_chunk, s->scal, (int)S_WNORM2, (const int*)s->ctrl, j, 1);
            }
            hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, st, s->ctrl, s->hcol, s->hcol2, s->H, s->cs,
                               s->sn, s->g, s->scal, mm + 1, mcyc);
            hipLaunchKernelGGL((normalize_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, (const P*)w, s->n,
                               s->ctrl, s->scal);
        }
        DG_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(trisolve_kernel, dim3(1), dim3(1024), 0, st, s->ctrl, s->H, s->g, s->y, mm + 1);
        pr = prof_begin(s, st, PK_COMBINE, 0.0, -2, 0);
        hipLaunchKernelGGL((combine_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, s->n, s->ctrl,
                           s->y, (P*)s->u);
        prof_end(s, st, pr);
        hipLaunchKernelGGL((dinv_update_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Dinv,
                           (const P*)s->u, x, s->T);
        DG_HIP_CHECK(hipGetLastError());
        rep->cycles++;
    }
    if (s->o.profile) prof_flush(s, 0, nullptr);
    rep->status = status;
    return status;
}

namespace dg {
// The solver no longer holds a matrix (its values were temporary): the next
// solve needs dg_solver_setup first.
void solver_invalidate(dg_solver* s)
{
    if (!s) return;
    s->ready = false;
    s->A64 = nullptr;
}
}  // namespace dg

extern "C" int32_t dg_solver_solve(dg_solver* s, const double* b, double* x, dg_solve_report* rep, void* stream)
{
    if (!s || !b || !x || !rep) return DG_ERR_ARG;
    if (!s->ready) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    *rep = dg_solve_report{};
    if (s->small) {
        SmallArgs a{};
        a.A64 = s->A64;
        a.rp = s->m->d_row_ptr;
        a.ci = s->m->d_col_idx;
        a.Ahat = s->Ahat;
        a.Dinv = s->Dinv;
        a.b = b;
        a.x = x;
        a.rep = s->h_rep;
        a.T = s->T;
        a.nnzb = (int32_t)s->m->nnzb;
        a.m = s->o.restart;
        a.max_iters = s->o.max_iters;
        a.mixed = s->mixed;
        a.rel_tol = s->o.rel_tol;
        a.inner_tol = s->o.inner_tol;
        a.guess_limit = s->o.guess_limit;
        a.L = s->sl;
        *s->h_rep = dg_solve_report{};
        s->h_rep->status = DG_ERR_HIP;  // stays if the kernel never ran
        const int r = small_launch(s->N, s->mixed, a, st);
        if (r != DG_OK) return r;
        DG_HIP_CHECK(hipStreamSynchronize(st));
        *rep = *s->h_rep;
        rep->persistent = 1;
        return rep->status;
    }
    int r;
    switch (s->N) {
    case 1: r = s->mixed ? solve_np<1, float>(s, b, x, rep, st) : solve_np<1, double>(s, b, x, rep, st); break;
    case 3: r = s->mixed ? solve_np<3, float>(s, b, x, rep, st) : solve_np<3, double>(s, b, x, rep, st); break;
    case 6: r = s->mixed ? solve_np<6, float>(s, b, x, rep, st) : solve_np<6, double>(s, b, x, rep, st); break;
    case 10: r = s->mixed ? solve_np<10, float>(s, b, x, rep, st) : solve_np<10, double>(s, b, x, rep, st); break;
    case 15: r = s->mixed ? solve_np<15, float>(s, b, x, rep, st) : solve_np<15, double>(s, b, x, rep, st); break;
    default: return DG_ERR_DEGREE;
    }
    rep->status = r;
    return r;
}

template <int N>
static int residual_n(const dg_mesh* m, const double* A, const double* b, const double* x, double* y, hipStream_t st)
{
    const int EPW = 64 / N;
    const int grid = (int)((m->T + 4 * EPW - 1) / (4 * EPW));
    hipLaunchKernelGGL((residual64_kernel<N>), dim3(grid), dim3(BLK), 0, st, A, m->d_row_ptr, m->d_col_idx, b, x, y,
                       m->T, (double*)nullptr);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_residual(const dg_mesh* m, const double* A, const double* b, const double* x, double* y,
                               void* stream)
{
    if (!m || !A || !x || !y) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    switch (m->n) {
    case 1: return residual_n<1>(m, A, b, x, y, st);
    case 3: return residual_n<3>(m, A, b, x, y, st);
    case 6: return residual_n<6>(m, A, b, x, y, st);
    case 10: return residual_n<10>(m, A, b, x, y, st);
    case 15: return residual_n<15>(m, A, b, x, y, st);
    }
    return DG_ERR_DEGREE;
}

extern "C" int32_t dg_solver_profile(dg_solver* s, dg_kernel_stats* out, int32_t max, int32_t* count, int32_t reset)
{
    if (!s || !count || (max > 0 && !out)) return DG_ERR_ARG;
    int c = 0;
    for (int k = 0; k < PK_N && c < max; ++k, ++c) {
        std::snprintf(out[c].name, sizeof(out[c].name), "%s", PK_NAMES[k]);
        out[c].launches = s->pl[k];
        out[c].ms = s->pms[k];
        out[c].bytes = s->pbytes[k];
    }
    *count = c;
    if (reset)
        for (int k = 0; k < PK_N; ++k) { s->pl[k] = 0; s->pms[k] = 0.0; s->pbytes[k] = 0.0; }
    return DG_OK;
}

extern "C" int32_t dg_solver_preconditioner(dg_solver* s, double* dinv64, void* ahat, void* stream)
{
    if (!s || !s->ready) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const size_t NN = (size_t)s->N * s->N;
    if (dinv64) DG_HIP_CHECK(hipMemcpyAsync(dinv64, s->Dinv64, sizeof(double) * NN * s->T, hipMemcpyDeviceToDevice, st));
    if (ahat && s->n_off > 0)
        DG_HIP_CHECK(hipMemcpyAsync(ahat, s->Ahat, (s->mixed ? sizeof(float) : sizeof(double)) * NN * s->n_off,
                                    hipMemcpyDeviceToDevice, st));
    return DG_OK;
}
