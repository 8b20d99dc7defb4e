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
#include <new>

#include "dg_internal.h"

namespace dg {

enum { C_J = 0, C_STOP = 1, C_REORTH = 2, C_TICKET0 = 4, C_NCTRL = 16 };
enum { S_BNORM2 = 0, S_RNORM2 = 1, S_INVH = 2, S_WNORM2 = 3, S_HN = 4, S_CYCTOL = 5, S_BETA = 6, S_NSCAL = 8 };

constexpr int BLK = 256;
constexpr int CHUNK_E = 4;                // vector entries per thread in the chunked kernels
constexpr int CHUNK = BLK * CHUNK_E;      // entries per block

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

// Block partials are published with a device-scope release; the block that
// draws the last ticket acquires them and reduces in fixed block order
// (deterministic), then resets the ticket for the next launch.
__device__ __forceinline__ bool last_block(int* ticket)
{
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        int t = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == (int)gridDim.x - 1);
        if (last) __threadfence();
    }
    __syncthreads();
    return last;
}

// ---------------------------------------------------------------------------
// FP64 residual y = b - A x (A = full BSR incl. diagonal blocks); lane per
// (element, row i).  Optionally accumulates ||y||^2 into scal[slot].
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(BLK) void residual64_kernel(const double* __restrict__ A, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const double* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int64_t T, double* partials, int* ticket, double* scal,
                                                         int slot)
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
    if (last_block(ticket)) {
        double acc = 0.0;
        for (int bl = threadIdx.x; bl < (int)gridDim.x; bl += BLK) acc += partials[bl];
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) { scal[slot] = acc; *ticket = 0; }
    }
}

// ||v||^2 of an FP64 vector into scal[slot]
__global__ __launch_bounds__(BLK) void norm2_kernel(const double* __restrict__ v, int64_t n, double* partials,
                                                    int* ticket, double* scal, int slot)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) acc += v[t] * v[t];
    const double bs = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(ticket)) {
        double a2 = 0.0;
        for (int bl = threadIdx.x; bl < (int)gridDim.x; bl += BLK) a2 += partials[bl];
        a2 = block_sum(a2, sh);
        if (threadIdx.x == 0) { scal[slot] = a2; *ticket = 0; }
    }
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
                                                       const int* __restrict__ ctrl)
{
    if (ctrl[C_STOP]) return;
    constexpr int EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = lane / N, i = lane - e * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e;
    if (e >= EPW || el >= T) return;
    const P* v = Vbase + (int64_t)ctrl[C_J] * n;
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

// h[i] = V_i . w for i = 0..j, and ||w||^2 (into hcol[j+1]); chunked over n.
template <typename P>
__global__ __launch_bounds__(BLK) void multidot_kernel(const P* __restrict__ V, const P* __restrict__ w, int64_t n,
                                                       int* ctrl, double* partials, int ldp, double* hcol,
                                                       int ticket_slot, int only_if_reorth)
{
    if (ctrl[C_STOP] || (only_if_reorth && !ctrl[C_REORTH])) return;
    __shared__ double sh[4];
    const int j = ctrl[C_J];
    const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
    double wr[CHUNK_E];
#pragma unroll
    for (int e = 0; e < CHUNK_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        wr[e] = t < n ? (double)w[t] : 0.0;
    }
    for (int i = 0; i <= j + 1; ++i) {
        double acc = 0.0;
        if (i <= j) {
            const P* vi = V + (int64_t)i * n;
#pragma unroll
            for (int e = 0; e < CHUNK_E; ++e) {
                const int64_t t = base + (int64_t)e * BLK;
                if (t < n) acc += (double)vi[t] * wr[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < CHUNK_E; ++e) acc += wr[e] * wr[e];
        }
        const double bs = block_sum(acc, sh);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * ldp + i] = bs;
    }
    if (last_block(ctrl + ticket_slot)) {
        for (int i = threadIdx.x; i <= j + 1; i += BLK) {
            double s = 0.0;
            for (int bl = 0; bl < (int)gridDim.x; ++bl) s += partials[(int64_t)bl * ldp + i];
            hcol[i] = s;
        }
        if (threadIdx.x == 0) ctrl[ticket_slot] = 0;
    }
}

// w -= sum_i h[i] V_i; ||w||^2 into scal[S_WNORM2]; in the reorthogonalisation
// pass (reorth != 0) it runs only when flagged and adds h2 into h.
template <typename P>
__global__ __launch_bounds__(BLK) void update_kernel(const P* __restrict__ V, P* __restrict__ w, int64_t n, int* ctrl,
                                                     double* partials, const double* hcol, double* scal,
                                                     int ticket_slot, int reorth_pass)
{
    if (ctrl[C_STOP] || (reorth_pass && !ctrl[C_REORTH])) return;
    __shared__ double sh[4];
    const int j = ctrl[C_J];
    const int64_t base = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
    double wr[CHUNK_E];
#pragma unroll
    for (int e = 0; e < CHUNK_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        wr[e] = t < n ? (double)w[t] : 0.0;
    }
    for (int i = 0; i <= j; ++i) {
        const double h = hcol[i];
        const P* vi = V + (int64_t)i * n;
#pragma unroll
        for (int e = 0; e < CHUNK_E; ++e) {
            const int64_t t = base + (int64_t)e * BLK;
            if (t < n) wr[e] -= h * (double)vi[t];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < CHUNK_E; ++e) {
        const int64_t t = base + (int64_t)e * BLK;
        if (t < n) {
            const P pv = (P)wr[e];
            w[t] = pv;
            acc += (double)pv * (double)pv;
        }
    }
    const double bs = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(ctrl + ticket_slot)) {
        double a2 = 0.0;
        for (int bl = threadIdx.x; bl < (int)gridDim.x; bl += BLK) a2 += partials[bl];
        a2 = block_sum(a2, sh);
        if (threadIdx.x == 0) {
            scal[S_WNORM2] = a2;
            ctrl[ticket_slot] = 0;
        }
    }
}

// One thread: reorthogonalisation decision (after the first pass) or the
// Hessenberg column, Givens rotations, residual estimate and stop flag.
__global__ void arnoldi_decide_kernel(int* ctrl, const double* hcol, double* scal, int want_reorth)
{
    if (ctrl[C_STOP]) return;
    const double before = hcol[ctrl[C_J] + 1];  // ||w||^2 before the first pass
    ctrl[C_REORTH] = (want_reorth && scal[S_WNORM2] < 0.5 * before) ? 1 : 0;
}

__global__ void givens_kernel(int* ctrl, double* hcol, const double* hcol2, double* H, double* cs, double* sn,
                              double* g, double* scal, int ldh, int mcyc)
{
    if (ctrl[C_STOP]) return;
    const int j = ctrl[C_J];
    const bool re = ctrl[C_REORTH] != 0;
    double* col = H + (int64_t)j * ldh;  // column-major: H[i + j*ldh]
    for (int i = 0; i <= j; ++i) col[i] = hcol[i] + (re ? hcol2[i] : 0.0);
    const double hn = sqrt(scal[S_WNORM2]);
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = hn;
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

// y = H(0:J,0:J)^{-1} g(0:J), one thread (H column-major, leading dimension ldh)
__global__ void trisolve_kernel(const int* ctrl, const double* H, const double* g, double* y, int ldh)
{
    const int J = ctrl[C_J];
    for (int i = J - 1; i >= 0; --i) {
        double s = g[i];
        for (int c = i + 1; c < J; ++c) s -= H[i + (int64_t)c * ldh] * y[c];
        y[i] = s / H[i + (int64_t)i * ldh];
    }
}

// u = V(:,0:J) y
template <typename P>
__global__ __launch_bounds__(BLK) void combine_kernel(const P* __restrict__ V, int64_t n, const int* ctrl,
                                                      const double* __restrict__ y, P* __restrict__ u)
{
    const int J = ctrl[C_J];
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLK) {
        double s = 0.0;
        for (int i = 0; i < J; ++i) s += y[i] * (double)V[(int64_t)i * n + t];
        u[t] = (P)s;
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
    double* H = nullptr;
    double* cs = nullptr;
    double* sn = nullptr;
    double* g = nullptr;
    double* y = nullptr;
    double* scal = nullptr;
    int* ctrl = nullptr;
    int* bad = nullptr;
    int ready = 0;
};

static void solver_free(dg_solver* s)
{
    hipFree(s->Ahat); hipFree(s->Dinv); hipFree(s->Dinv64); hipFree(s->V); hipFree(s->w); hipFree(s->u);
    hipFree(s->r); hipFree(s->partials); hipFree(s->hcol); hipFree(s->hcol2); hipFree(s->H); hipFree(s->cs);
    hipFree(s->sn); hipFree(s->g); hipFree(s->y); hipFree(s->scal); hipFree(s->ctrl); hipFree(s->bad);
}

extern "C" int32_t dg_solver_create(const dg_mesh* m, const dg_solver_opts* o, dg_solver** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (!m || !o) return DG_ERR_ARG;
    if (o->restart < 1 || o->restart > 4096 || o->max_iters < 0 || !(o->rel_tol > 0) || (o->mixed != 0 && o->mixed != 1))
        return DG_ERR_ARG;
    if (o->mixed && !(o->inner_tol > 0 && o->inner_tol < 1)) return DG_ERR_ARG;
    dg_solver* s = new (std::nothrow) dg_solver();
    if (!s) return DG_ERR_OOM;
    s->m = m;
    s->o = *o;
    s->N = m->n;
    s->T = m->T;
    s->n = m->T * m->n;
    s->n_off = m->nnzb - m->T;
    s->mixed = o->mixed;
    const int EPW = 64 / s->N;
    s->grid_elem = (int)((s->T + 4 * EPW - 1) / (4 * EPW));
    s->grid_chunk = (int)((s->n + CHUNK - 1) / CHUNK);
    s->grid_vec = (int)std::min<int64_t>((s->n + BLK - 1) / BLK, 2048);
    const size_t ps = s->mixed ? sizeof(float) : sizeof(double);
    const int mm = o->restart;
    const size_t NN = (size_t)s->N * s->N;
    const int maxgrid = std::max(std::max(s->grid_elem, s->grid_chunk), s->grid_vec);
    bool ok = true;
    auto al = [&](void** p, size_t bytes) { if (ok && hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) { *p = nullptr; ok = false; } };
    al(&s->Ahat, ps * NN * std::max<int64_t>(s->n_off, 1));
    al(&s->Dinv, ps * NN * s->T);
    al((void**)&s->Dinv64, sizeof(double) * NN * s->T);
    al(&s->V, ps * (size_t)(mm + 1) * s->n);
    al(&s->w, ps * s->n);
    al(&s->u, ps * s->n);
    al((void**)&s->r, sizeof(double) * s->n);
    al((void**)&s->partials, sizeof(double) * (size_t)maxgrid * (mm + 2));
    al((void**)&s->hcol, sizeof(double) * (mm + 2));
    al((void**)&s->hcol2, sizeof(double) * (mm + 2));
    al((void**)&s->H, sizeof(double) * (size_t)(mm + 1) * mm);
    al((void**)&s->cs, sizeof(double) * mm);
    al((void**)&s->sn, sizeof(double) * mm);
    al((void**)&s->g, sizeof(double) * (mm + 1));
    al((void**)&s->y, sizeof(double) * mm);
    al((void**)&s->scal, sizeof(double) * S_NSCAL);
    al((void**)&s->ctrl, sizeof(int) * C_NCTRL);
    al((void**)&s->bad, sizeof(int));
    if (!ok) { solver_free(s); delete s; return DG_ERR_OOM; }
    if (hipMemset(s->ctrl, 0, sizeof(int) * C_NCTRL) != hipSuccess) { solver_free(s); delete s; return DG_ERR_HIP; }
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
    const int ldp = mm + 2;
    P* V = (P*)s->V;
    P* w = (P*)s->w;
    // ||b||
    hipLaunchKernelGGL(norm2_kernel, dim3(s->grid_vec), dim3(BLK), 0, st, b, s->n, s->partials, s->ctrl + C_TICKET0,
                       s->scal, (int)S_BNORM2);
    DG_HIP_CHECK(hipGetLastError());
    double hs[S_NSCAL];
    int hc[C_NCTRL];
    DG_HIP_CHECK(hipMemcpyAsync(hs, s->scal, sizeof(hs), hipMemcpyDeviceToHost, st));
    DG_HIP_CHECK(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(hs[S_BNORM2]);
    if (!std::isfinite(bnorm)) return DG_ERR_NONFINITE;
    rep->iters = 0;
    rep->cycles = 0;
    rep->rel_res0 = 0.0;
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
    for (;;) {
        hipLaunchKernelGGL((residual64_kernel<N>), dim3(s->grid_elem), dim3(BLK), 0, st, s->A64, m->d_row_ptr,
                           m->d_col_idx, b, x, s->r, s->T, s->partials, s->ctrl + C_TICKET0 + 1, s->scal,
                           (int)S_RNORM2);
        DG_HIP_CHECK(hipGetLastError());
        DG_HIP_CHECK(hipMemcpyAsync(hs, s->scal, sizeof(hs), hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipMemcpyAsync(hc, s->ctrl, sizeof(hc), hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipStreamSynchronize(st));
        if (rep->cycles > 0) its += hc[C_J];
        const double rel = std::sqrt(hs[S_RNORM2]) / bnorm;
        if (rep->cycles == 0) rep->rel_res0 = rel;
        rep->rel_res = rel;
        rep->iters = its;
        if (!std::isfinite(rel)) { status = DG_ERR_NONFINITE; break; }
        if (rel <= s->o.rel_tol) { status = DG_OK; break; }
        if (its >= s->o.max_iters) { status = DG_NOT_CONVERGED; break; }
        const int mcyc = std::min(mm, s->o.max_iters - its);
        hipLaunchKernelGGL((cycle_init_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, s->r, s->n, s->ctrl,
                           s->scal, s->g, cyc_rel, abs_tol);
        for (int j = 0; j < mcyc; ++j) {
            hipLaunchKernelGGL((spmv_hat_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Ahat,
                               m->d_row_ptr, m->d_col_idx, (const P*)V, s->n, w, s->T, s->ctrl);
            hipLaunchKernelGGL((multidot_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V,
                               (const P*)w, s->n, s->ctrl, s->partials, ldp, s->hcol, (int)C_TICKET0 + 2, 0);
            hipLaunchKernelGGL((update_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, w, s->n,
                               s->ctrl, s->partials, s->hcol, s->scal, (int)C_TICKET0 + 3, 0);
            if (s->o.reorth) {
                hipLaunchKernelGGL(arnoldi_decide_kernel, dim3(1), dim3(1), 0, st, s->ctrl, s->hcol, s->scal, 1);
                hipLaunchKernelGGL((multidot_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V,
                                   (const P*)w, s->n, s->ctrl, s->partials, ldp, s->hcol2, (int)C_TICKET0 + 2, 1);
                hipLaunchKernelGGL((update_kernel<P>), dim3(s->grid_chunk), dim3(BLK), 0, st, (const P*)V, w, s->n,
                                   s->ctrl, s->partials, s->hcol2, s->scal, (int)C_TICKET0 + 3, 1);
            }
            hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(1), 0, st, s->ctrl, s->hcol, s->hcol2, s->H, s->cs, s->sn,
                               s->g, s->scal, mm + 1, mcyc);
            hipLaunchKernelGGL((normalize_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, V, (const P*)w, s->n,
                               s->ctrl, s->scal);
        }
        DG_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(trisolve_kernel, dim3(1), dim3(1), 0, st, s->ctrl, s->H, s->g, s->y, mm + 1);
        hipLaunchKernelGGL((combine_kernel<P>), dim3(s->grid_vec), dim3(BLK), 0, st, (const P*)V, s->n, s->ctrl, s->y,
                           (P*)s->u);
        hipLaunchKernelGGL((dinv_update_kernel<N, P>), dim3(s->grid_elem), dim3(BLK), 0, st, (const P*)s->Dinv,
                           (const P*)s->u, x, s->T);
        DG_HIP_CHECK(hipGetLastError());
        rep->cycles++;
    }
    rep->status = status;
    return status;
}

extern "C" int32_t dg_solver_solve(dg_solver* s, const double* b, double* x, dg_solve_report* rep, void* stream)
{
    if (!s || !b || !x || !rep) return DG_ERR_ARG;
    if (!s->ready) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    *rep = dg_solve_report{};
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
                       m->T, (double*)nullptr, (int*)nullptr, (double*)nullptr, 0);
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
