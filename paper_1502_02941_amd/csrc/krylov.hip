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

namespace dg {

enum { C_J = 0, C_STOP = 1, C_REORTH = 2, C_NREORTH = 3, C_NCTRL = 16 };
enum { S_BNORM2 = 0, S_RNORM2 = 1, S_INVH = 2, S_WNORM2 = 3, S_HN = 4, S_CYCTOL = 5, S_BETA = 6,
       S_Q1 = 7, S_Q2A = 8, S_Q2B = 9, S_NSCAL = 12 };

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
// w = v + sum_L Ahat_KL v_L ; lane per (element, row i)
template <int N, typename P>
__global__ __launch_bounds__(BLK) void spmv_hat_kernel(const P* __restrict__ Ahat, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const P* __restrict__ Vbase,
                                                       int64_t n, P* __restrict__ w, int64_t T,
                                                       const int* __restrict__ ctrl, const P* __restrict__ vin)
{
    if (ctrl[C_STOP]) return;
    constexpr int EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e;
    if (e >= EPW || el >= T) return;
    const P* v = vin ? vin : Vbase + (int64_t)ctrl[C_J] * n;  // vin: the block's second product
    const int s0 = rp[el], s1 = rp[el + 1];
    const int64_t c0 = (int64_t)s0 - el;
    P s = v[el * N + i];
    for (int sl = s0 + 1; sl < s1; ++sl) {
        const P* blk = Ahat + ((c0 + (sl - s0 - 1)) * N + i) * N;
        const P* xv = v + (int64_t)ci[sl] * N;
#pragma unroll
        for (int c = 0; c < N; ++c) s += blk[c] * xv[c];
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
// Two-vector Arnoldi blocks.  From the last basis vector v_j a block forms
// w0 = Ahat v_j and w1 = Ahat w0, projects both against v_0..v_j with one pass
// over the basis (R = V^T [w0 w1]) and updates them with a second pass
// (U = [w0 w1] - V R, with the 2 x 2 Gram matrix U^T U), so the basis is read
// twice per two Arnoldi steps instead of twice per step.  The Cholesky factor
// (r11, r12; r22) of the Gram matrix turns U into v_{j+1}, v_{j+2}, and the
// Hessenberg columns follow from Ahat v_j = w0 = V R_0 + r11 v_{j+1} and
// Ahat v_{j+1} = (w1 - Ahat V R_0) / r11 with Ahat V = V H.
// ---------------------------------------------------------------------------

// partial V_c . w_r (c = 0..j, r = 0, 1), stored at partials[(r (j+1) + c) splits + split].
// Tiles of CT2 = 8 columns (measured on 786432 unknowns: 8 columns and 4096
// target blocks took 14% less time over a cycle than 16 columns and 2048).
constexpr int CT2 = 8;
constexpr int MD2_TARGET_BLOCKS = 4096;
template <typename P>
__global__ __launch_bounds__(BLK) void multidot2_kernel(const P* __restrict__ V, const P* __restrict__ w0,
                                                        const P* __restrict__ w1, int64_t n, int j,
                                                        int64_t rows_per_split, const int* ctrl,
                                                        double* __restrict__ partials)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    __shared__ double sh[4][2 * CT2];
    const int ncols = j + 1;
    const int c0 = blockIdx.x * CT2;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;
    const P* col[CT2];
#pragma unroll
    for (int c = 0; c < CT2; ++c) col[c] = (c0 + c < ncols) ? V + (int64_t)(c0 + c) * n : w0;  // past j: discarded
    double a0[CT2], a1[CT2];
#pragma unroll
    for (int c = 0; c < CT2; ++c) a0[c] = a1[c] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BLK) {
        const double x0 = (double)w0[r], x1 = (double)w1[r];
#pragma unroll
        for (int c = 0; c < CT2; ++c) {
            const double v = (double)col[c][r];
            a0[c] += v * x0;
            a1[c] += v * x1;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CT2; ++c) {
        const double v0 = wave_sum(a0[c]), v1 = wave_sum(a1[c]);
        if (lane == 0) {
            sh[wave][c] = v0;
            sh[wave][CT2 + c] = v1;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * CT2) {
        const int rr = threadIdx.x / CT2, c = threadIdx.x - rr * CT2;
        if (c0 + c < ncols)
            partials[((int64_t)rr * ncols + c0 + c) * gridDim.y + blockIdx.y] =
                (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    }
}

// w_r -= sum_{c<=j} R[r][c] V_c for r = 0, 1 (R = [R_0 | R_1], each j+1 long),
// and the Gram partials of the results: partials[k * gridDim.x + block] for
// k = 0: u0.u0, 1: u0.u1, 2: u1.u1
template <typename P>
__global__ __launch_bounds__(BLK) void update2_kernel(const P* __restrict__ V, P* __restrict__ w0, P* __restrict__ w1,
                                                      int64_t n, int j, const int* ctrl, double* partials,
                                                      const double* __restrict__ R)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    __shared__ double sh[4];
    const double* R0 = R;
    const double* R1 = R + (j + 1);
    const int64_t base = (int64_t)blockIdx.x * (BLK * UPD_E) + threadIdx.x;
    double u0[UPD_E], u1[UPD_E];
    bool in[UPD_E];
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        in[e] = t < n;
        u0[e] = in[e] ? (double)w0[t] : 0.0;
        u1[e] = in[e] ? (double)w1[t] : 0.0;
    }
    int c = 0;
    for (; c + 3 <= j; c += 4) {
        const double p0 = R0[c], p1 = R0[c + 1], p2 = R0[c + 2], p3 = R0[c + 3];
        const double q0 = R1[c], q1 = R1[c + 1], q2 = R1[c + 2], q3 = R1[c + 3];
        const P* v0 = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e]) {
                const double a = (double)v0[t], b = (double)v0[t + n], cc = (double)v0[t + 2 * n],
                             d = (double)v0[t + 3 * n];
                u0[e] -= p0 * a + p1 * b + p2 * cc + p3 * d;
                u1[e] -= q0 * a + q1 * b + q2 * cc + q3 * d;
            }
        }
    }
    for (; c <= j; ++c) {
        const double p0 = R0[c], q0 = R1[c];
        const P* vc = V + (int64_t)c * n;
#pragma unroll
        for (int e = 0; e < UPD_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (in[e]) {
                const double a = (double)vc[t];
                u0[e] -= p0 * a;
                u1[e] -= q0 * a;
            }
        }
    }
    double g00 = 0.0, g01 = 0.0, g11 = 0.0;
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
        if (in[e]) {
            const int64_t t = base + (int64_t)e * BLK;
            const P a = (P)u0[e], b = (P)u1[e];
            w0[t] = a;
            w1[t] = b;
            g00 += (double)a * (double)a;
            g01 += (double)a * (double)b;
            g11 += (double)b * (double)b;
        }
    }
    const double s00 = block_sum(g00, sh);
    const double s01 = block_sum(g01, sh);
    const double s11 = block_sum(g11, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s00;
        partials[gridDim.x + blockIdx.x] = s01;
        partials[2 * gridDim.x + blockIdx.x] = s11;
    }
}

// One workgroup: Gram reduction, Cholesky, Hessenberg columns j and j+1 (raw
// copies in Hr, leading dimension ldr; rotated in H, leading dimension ldh),
// the previous Givens rotations applied to them in turn, the new rotations,
// residual estimates and stop tests.  Column j+1 is taken only when column j
// did not stop the cycle; when r22 is not resolvable (the second vector lies
// in the span to working accuracy) the cycle stops after column j+1.
constexpr int BG_T = 1024;
__device__ void bg_rotate(double* colv, int count, const double* __restrict__ cs, const double* __restrict__ sn,
                          double* sc, double* ss)
{
    double a = colv[0];
    for (int i0 = 0; i0 < count; i0 += GV_CHUNK) {
        const int cnt = count - i0 < GV_CHUNK ? count - i0 : GV_CHUNK;
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += BG_T) {
            sc[t] = cs[i0 + t];
            ss[t] = sn[i0 + t];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int t = 0; t < cnt; ++t) {
                const double b = colv[i0 + t + 1];
                colv[i0 + t] = sc[t] * a + ss[t] * b;
                a = -ss[t] * a + sc[t] * b;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) colv[count] = a;
    __syncthreads();
}

__global__ __launch_bounds__(BG_T) void block_givens_kernel(int* ctrl, const double* __restrict__ gp, int nparts,
                                                            const double* __restrict__ R, double* __restrict__ Hr,
                                                            int ldr, double* __restrict__ H, int ldh,
                                                            double* __restrict__ cs, double* __restrict__ sn,
                                                            double* __restrict__ g, double* scal, int j, int mcyc)
{
    if (ctrl[C_STOP] || ctrl[C_J] != j) return;
    __shared__ double red[3][BG_T / 64];
    __shared__ double colA[TS_MAXJ + 4], colB[TS_MAXJ + 4];
    __shared__ double sc[GV_CHUNK], ss[GV_CHUNK];
    __shared__ double fac[3];
    __shared__ int take2, stop1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double a00 = 0.0, a01 = 0.0, a11 = 0.0;
    for (int t = threadIdx.x; t < nparts; t += BG_T) {
        a00 += gp[t];
        a01 += gp[nparts + t];
        a11 += gp[2 * nparts + t];
    }
    a00 = wave_sum(a00);
    a01 = wave_sum(a01);
    a11 = wave_sum(a11);
    if (lane == 0) {
        red[0][wave] = a00;
        red[1][wave] = a01;
        red[2][wave] = a11;
    }
    const double* R0 = R;
    const double* R1 = R + (j + 1);
    for (int i = threadIdx.x; i <= j; i += BG_T) colA[i] = R0[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double G00 = 0.0, G01 = 0.0, G11 = 0.0;
        for (int w = 0; w < BG_T / 64; ++w) {
            G00 += red[0][w];
            G01 += red[1][w];
            G11 += red[2][w];
        }
        const double r11 = sqrt(G00);
        const bool brk1 = !(r11 > 1e-300) || !isfinite(r11);
        const double r12 = brk1 ? 0.0 : G01 / r11;
        const double d = G11 - r12 * r12;
        const double r22 = d > 0.0 ? sqrt(d) : 0.0;
        const bool ok2 = !brk1 && isfinite(r22) && r22 > 1e-8 * sqrt(G11);
        fac[0] = r11;
        fac[1] = r12;
        fac[2] = r22;
        colA[j + 1] = r11;
        scal[S_Q1] = brk1 ? 0.0 : 1.0 / r11;
        scal[S_Q2A] = ok2 ? 1.0 / r22 : 0.0;
        scal[S_Q2B] = ok2 ? -r12 / (r11 * r22) : 0.0;
        scal[S_HN] = r11;
        take2 = ok2 ? 1 : 0;
        stop1 = brk1 ? 1 : 0;
    }
    __syncthreads();
    // raw column j
    for (int i = threadIdx.x; i <= j + 1; i += BG_T) Hr[i + (int64_t)j * ldr] = colA[i];
    __syncthreads();
    // raw column j+1 (before colA is rotated): (R_1 + r12 e_{j+1} + r22 e_{j+2} - Hr(0:j+1, 0:j) R_0) / r11
    const bool want2 = !stop1 && j + 1 < mcyc;
    if (want2) {
        const double r11 = fac[0];
        for (int i = threadIdx.x; i <= j + 1; i += BG_T) {
            double t = 0.0;
            for (int c = i > 0 ? i - 1 : 0; c <= j; ++c) t += Hr[i + (int64_t)c * ldr] * R0[c];
            const double base = i <= j ? R1[i] : fac[1];
            colB[i] = (base - t) / r11;
        }
        if (threadIdx.x == 0) colB[j + 2] = fac[2] / r11;
        __syncthreads();
        for (int i = threadIdx.x; i <= j + 2; i += BG_T) Hr[i + (int64_t)(j + 1) * ldr] = colB[i];
    }
    // column j: previous rotations, new rotation, estimate
    bg_rotate(colA, j, cs, sn, sc, ss);
    if (threadIdx.x == 0) {
        const double a = colA[j], b = colA[j + 1];
        const double d = sqrt(a * a + b * b);
        cs[j] = d == 0.0 ? 1.0 : a / d;
        sn[j] = d == 0.0 ? 0.0 : b / d;
        colA[j] = d;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        const bool stop = stop1 || fabs(g[j + 1]) <= scal[S_CYCTOL] || j + 1 >= mcyc;
        if (stop) stop1 = 1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += BG_T) H[i + (int64_t)j * ldh] = colA[i];
    if (stop1 || !want2) {
        if (threadIdx.x == 0) {
            ctrl[C_J] = j + 1;
            ctrl[C_REORTH] = 0;
            ctrl[C_STOP] = 1;
        }
        return;
    }
    // column j+1
    bg_rotate(colB, j + 1, cs, sn, sc, ss);
    if (threadIdx.x == 0) {
        const int k = j + 1;
        const double a = colB[k], b = colB[k + 1];
        const double d = sqrt(a * a + b * b);
        cs[k] = d == 0.0 ? 1.0 : a / d;
        sn[k] = d == 0.0 ? 0.0 : b / d;
        colB[k] = d;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        ctrl[C_J] = k + 1;
        ctrl[C_REORTH] = 0;
        if (!take2 || fabs(g[k + 1]) <= scal[S_CYCTOL] || k + 1 >= mcyc) ctrl[C_STOP] = 1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += BG_T) H[i + (int64_t)(j + 1) * ldh] = colB[i];
}

// v_{j+1} = u0 / r11 and v_{j+2} = u1 / r22 - r12 / (r11 r22) u0, each when the
// block took its column (ctrl[C_J] already advanced by the block kernel)
template <typename P>
__global__ __launch_bounds__(BLK) void normalize2_kernel(P* __restrict__ V, const P* __restrict__ w0,
                                                         const P* __restrict__ w1, int64_t n, int j, const int* ctrl,
                                                         const double* scal)
{
    const int J = ctrl[C_J];
    if (J != j + 2) return;  // the block took only column j (the cycle stopped there) or did not run
    const bool second = !ctrl[C_STOP];
    const double a = scal[S_Q1], b = scal[S_Q2A], c = scal[S_Q2B];
    P* o1 = V + (int64_t)(j + 1) * n;
    P* o2 = V + (int64_t)(j + 2) * n;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        const double u0 = (double)w0[t];
        o1[t] = (P)(u0 * a);
        if (second) o2[t] = (P)((double)w1[t] * b + u0 * c);
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
            for (int c = 0; c < pb; ++c) s -= H[k + (int64_t)(c0 + c) * ldh] * ys[c];
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
    double* r = nullptr;    // [n] FP64
    double* partials = nullptr;
    double* hcol = nullptr;
    double* hcol2 = nullptr;
    double* Rb = nullptr;   // [2][restart + 2]: a two-vector block's projections
    double* Hr = nullptr;   // [restart + 1][restart + 2]: raw Hessenberg columns of the block path
    int block = 1;          // Arnoldi vectors per Gram-Schmidt pass (1 or 2)
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
    struct Rec { int cls; double bytes; int j; int pass; hipEvent_t e0, e1; };
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<Rec> pending;
    int64_t pl[8] = {0};
    double pms[8] = {0}, pbytes[8] = {0};
    // multidot split for iteration j: (column tiles, row splits, rows per split)
    void md_shape(int j, int* tiles, int* splits, int64_t* rows) const;
    // the same for the two-vector block starting at column j
    void md_shape2(int j, int* tiles, int* splits, int64_t* rows) const;
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

void dg_solver::md_shape2(int j, int* tiles, int* splits, int64_t* rows) const
{
    const int nt = (j + 1 + dg::CT2 - 1) / dg::CT2;
    const int64_t max_splits = std::max<int64_t>(1, n / dg::MD_MIN_ROWS);
    int64_t sp = (dg::MD2_TARGET_BLOCKS + nt - 1) / nt;
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
static bool prof_begin(dg_solver* s, hipStream_t st, int cls, double bytes, int j, int pass)
{
    if (!s->o.profile) return false;
    dg_solver::Rec r{cls, bytes, j, pass, prof_event(s), prof_event(s)};
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
        s->pl[r.cls]++;
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
    hipFree(s->Rb); hipFree(s->Hr);
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
    if (o->persistent < -1 || o->persistent > 1) return DG_ERR_ARG;
    if (o->block < 0 || o->block > 2 || (o->block == 2 && o->reorth)) return DG_ERR_ARG;
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
    s->block = o->block == 0 ? (o->reorth ? 1 : 2) : o->block;
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
        s->md_shape2(j, &nt, &sp, &rows);
        maxgrid = std::max<int64_t>(maxgrid, (int64_t)sp * (j + 1) * 2);
    }
    maxgrid = std::max<int64_t>(maxgrid, 3 * (int64_t)s->grid_chunk);
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
    al((void**)&s->hcol, sizeof(double) * (mm + 2));
    al((void**)&s->hcol2, sizeof(double) * (mm + 2));
    if (s->block == 2) {
        al((void**)&s->Rb, sizeof(double) * 2 * (size_t)(mm + 2));
        al((void**)&s->Hr, sizeof(double) * (size_t)(mm + 2) * (mm + 1));
    }
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

template <int N>
static int setup_n(dg_solver* s, hipStream_t st)
{
    const dg_mesh* m = s->m;
    DG_HIP_CHECK(hipMemsetAsync(s->bad, 0, sizeof(int), st));
    constexpr int TPB = inv_tpb<N>();
    hipLaunchKernelGGL((invert_diag_kernel<N>), dim3((unsigned)((s->T + TPB - 1) / TPB)), dim3(TPB), 0, st, s->A64,
                       m->d_row_ptr, s->T, s->Dinv64, s->bad);
    DG_HIP_CHECK(hipGetLastError());
    if (s->mixed)
        hipLaunchKernelGGL((form_ahat_kernel<N, float>), dim3(s->grid_elem), dim3(BLK), 0, st, s->A64, m->d_row_ptr,
                           m->d_col_idx, s->Dinv64, s->T, (float*)s->Ahat, (float*)s->Dinv);
    else
        hipLaunchKernelGGL((form_ahat_kernel<N, double>), dim3(s->grid_elem), dim3(BLK), 0, st, s->A64, m->d_row_ptr,
                           m->d_col_idx, s->Dinv64, s->T, (double*)s->Ahat, (double*)s->Dinv);
    DG_HIP_CHECK(hipGetLastError());
    int bad = 0;
    DG_HIP_CHECK(hipMemcpyAsync(&bad, s->bad, sizeof(int), hipMemcpyDeviceToHost, st));
    DG_HIP_CHECK(hipStreamSynchronize(st));
    return bad ? DG_ERR_NONFINITE : DG_OK;
}

extern "C" int32_t dg_solver_setup(dg_solver* s, const double* A64, void* stream)
{
    if (!s || !A64) return DG_ERR_ARG;
    s->A64 = A64;
    s->ready = 0;
    hipStream_t st = (hipStream_t)stream;
    int r;
    switch (s->N) {
    case 1: r = setup_n<1>(s, st); break;
    case 3: r = setup_n<3>(s, st); break;
    case 6: r = setup_n<6>(s, st); break;
    case 10: r = setup_n<10>(s, st); break;
    case 15: r = setup_n<15>(s, st); break;
    default: return DG_ERR_DEGREE;
    }
    if (r == DG_OK) s->ready = 1;
    return r;
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
        if (s->o.profile) prof_flush(s, rep->cycles > 0 ? hc[C_J] : 0, s->o.reorth ? hflags.data() : nullptr);
        if (rep->cycles > 0) its += hc[C_J];
        const double rel = std::sqrt(hs[S_RNORM2]) / bnorm;
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
        hipLaunchKernelGGL((cycle_init_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, s->r, s->n, s->ctrl,
                           s->scal, s->g, cyc_rel, abs_tol);
        const double spmv_bytes = (double)s->n_off * N * N * ps + 2.0 * nb * ps + idx_bytes;
        P* w1 = (P*)s->u;  // the block's second vector (u is free until the cycle's combine)
        for (int j = 0; s->block == 2 && j < mcyc; j += 2) {
            int nt, sp;
            int64_t rows;
            s->md_shape2(j, &nt, &sp, &rows);
            const double md_bytes = (j + 3.0) * nb * ps, up_bytes = (j + 5.0) * nb * ps;
            pr = prof_begin(s, st, PK_SPMV, spmv_bytes, j, 0);
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Ahat,
                               m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, w, s->T, s->ctrl, (const P*)nullptr);
            prof_end(s, st, pr);
            pr = prof_begin(s, st, PK_SPMV, spmv_bytes, j, 0);
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Ahat,
                               m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, w1, s->T, s->ctrl, (const P*)w);
            prof_end(s, st, pr);
            pr = prof_begin(s, st, PK_MULTIDOT, md_bytes, j, 0);
            hipLaunchKernelGGL((multidot2_kernel<P>), dim3(nt, sp), dim3(BLK), 0, st, (const P*)V, (const P*)w,
                               (const P*)w1, s->n, j, rows, (const int*)s->ctrl, s->partials);
            prof_end(s, st, pr);
            hipLaunchKernelGGL(reduce_cols_kernel, dim3((2 * (j + 1) + 3) / 4), dim3(BLK), 0, st,
                               (const double*)s->partials, 2 * (j + 1), sp, j, (const int*)s->ctrl, s->Rb, 0);
            pr = prof_begin(s, st, PK_UPDATE, up_bytes, j, 0);
            hipLaunchKernelGGL((update2_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, w, w1, s->n, j,
                               (const int*)s->ctrl, s->partials, (const double*)s->Rb);
            prof_end(s, st, pr);
            hipLaunchKernelGGL(block_givens_kernel, dim3(1), dim3(BG_T), 0, st, s->ctrl, (const double*)s->partials,
                               s->grid_chunk, (const double*)s->Rb, s->Hr, mm + 2, s->H, mm + 1, s->cs, s->sn, s->g,
                               s->scal, j, mcyc);
            hipLaunchKernelGGL((normalize2_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, (const P*)w,
                               (const P*)w1, s->n, j, (const int*)s->ctrl, (const double*)s->scal);
        }
        for (int j = 0; s->block == 1 && j < mcyc; ++j) {
            int nt, sp;
            int64_t rows;
            s->md_shape(j, &nt, &sp, &rows);
            const double md_bytes = (j + 2.0) * nb * ps, up_bytes = (j + 3.0) * nb * ps;
            pr = prof_begin(s, st, PK_SPMV, spmv_bytes, j, 0);
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Ahat,
                               m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, w, s->T, s->ctrl, (const P*)nullptr);
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
