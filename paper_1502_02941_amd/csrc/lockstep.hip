// Lockstep batched block-Jacobi GMRES (gfx950).
//
// Solves many assembled instances together: every Arnoldi step is one launch
// per kernel covering all instances that are still iterating, so the whole GPU
// works on whatever is active and instances of very different cost need no
// load balancing.  Kernel boundaries order the steps (no inter-workgroup
// waiting).  Each launch maps its blocks to (instance, element block) or
// (instance, row chunk) through per-instance prefix offsets (binary search).
// Per instance, the method is the restarted GMRES of the single-mesh solver:
// FP64 true residual before every cycle, Arnoldi on A D^{-1} (identity
// diagonal blocks not stored) with classical Gram-Schmidt in precision P,
// Givens rotations, x += D^{-1} V y in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "dg_internal.h"
#include "lockstep.h"

namespace dg {

constexpr int LS_BT = 256;       // threads per block
constexpr int LS_CH = 1024;      // rows per row chunk (one workgroup each); measured fastest of 512..16384
constexpr int LS_CT = 16;        // Gram-Schmidt columns reduced together (8: same, 32: slower)
constexpr int LS_GV = 512;       // Givens staging chunk
constexpr int LS_BATCH = 8;      // loads issued together in the serial loops of the block kernels

__device__ __forceinline__ double ls_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ double ls_block_sum(double v, double* sh)
{
    v = ls_wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < LS_BT / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// last index i with pre[i] <= b (pre ascending, pre[0] = 0)
__device__ __forceinline__ int ls_find(const int64_t* __restrict__ pre, int count, int64_t b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool ls_running(const LsState& s) { return s.active && !s.stop; }

// Gauss-Jordan inverse with partial pivoting of an N x N block held by N
// lanes (row r in m[]); pivots found / broadcast with shuffles, interchanges
// as relabelling.  The lane labelled lr ends with row lr of the inverse.
template <int N>
__device__ __forceinline__ bool ls_invert_rows(double (&m)[N], const int r, const int gb, int& lr)
{
    lr = r;
    int pc[N];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double best = -1.0;
        int bl = 0, blabel = N, holder = 0;
#pragma unroll
        for (int t = 0; t < N; ++t) {
            const double v = fabs(__shfl(m[c], gb + t, 64));
            const int lt = __shfl(lr, gb + t, 64);
            if (lt >= c && (v > best || (v == best && lt < blabel))) { best = v; bl = t; blabel = lt; }
            if (lt == c) holder = t;
        }
        pc[c] = blabel;
        if (!(best > 0.0) || !isfinite(best)) ok = false;
        if (r == bl) lr = c;
        else if (r == holder) lr = blabel;
        double pr[N];
#pragma unroll
        for (int q = 0; q < N; ++q) pr[q] = __shfl(m[q], gb + bl, 64);
        const double inv = ok ? 1.0 / pr[c] : 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) pr[q] *= inv;
        pr[c] = inv;
        if (r == bl) {
#pragma unroll
            for (int q = 0; q < N; ++q) m[q] = pr[q];
        } else {
            const double f = m[c];
#pragma unroll
            for (int q = 0; q < N; ++q) m[q] -= f * pr[q];
            m[c] = -f * inv;
        }
    }
#pragma unroll
    for (int c = N - 1; c >= 0; --c) {
#pragma unroll
        for (int q = c + 1; q < N; ++q) {
            const bool sw = pc[c] == q;
            const double a = m[c], b = m[q];
            m[c] = sw ? b : a;
            m[q] = sw ? a : b;
        }
    }
    return ok;
}

// element-block mapping: returns false if this lane has no element
struct ElemLane {
    int inst;
    int64_t el;
    int j;
    int n;  // n_loc
};

__device__ __forceinline__ bool ls_elem_lane(const LsArgs& A, ElemLane& e)
{
    const int64_t b = blockIdx.x;
    e.inst = ls_find(A.eblk, A.count, b);
    const LsInst& I = A.inst[e.inst];
    e.n = (I.k + 1) * (I.k + 2) / 2;
    const int epw = 64 / e.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ein = lane / e.n;
    e.j = lane - ein * e.n;
    e.el = ((b - A.eblk[e.inst]) * (LS_BT / 64) + wave) * epw + ein;
    return ein < epw && e.el < I.T;
}

// ---------------------------------------------------------------------------
// setup: inverse diagonal blocks (FP64), then A D^{-1} and D^{-1} in P
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void ls_invert_one(const LsArgs& A, const LsInst& I, int64_t el, int j, bool act,
                                              int gb)
{
    const int32_t* rp = A.row_ptr + I.rp_off;
    const double* D = A.A64 + I.val_off + ((int64_t)(act ? rp[el] : 0) * N + j) * N;
    double m[N];
#pragma unroll
    for (int q = 0; q < N; ++q) m[q] = act ? D[q] : (q == j ? 1.0 : 0.0);
    int lr;
    const bool ok = ls_invert_rows<N>(m, j, gb, lr);
    if (act) {
        if (!ok) A.state[I.id_local].status = DG_ERR_NONFINITE;
        double* o = A.Dinv64 + I.dinv_off + (el * N + lr) * N;
#pragma unroll
        for (int q = 0; q < N; ++q) o[q] = m[q];
    }
}

__global__ __launch_bounds__(LS_BT) void ls_invert_kernel(const LsArgs A)
{
    ElemLane e;
    const bool act = ls_elem_lane(A, e);
    const LsInst& I = A.inst[e.inst];
    const int lane = threadIdx.x & 63;
    const int gb = (lane / e.n) * e.n;
    if (gb + e.n > 64) return;  // lanes past the last whole group of the wavefront
    if (I.k == 1) ls_invert_one<3>(A, I, e.el, e.j, act, gb);
    else ls_invert_one<6>(A, I, e.el, e.j, act, gb);
}

template <typename P, int N>
__device__ __forceinline__ void ls_form_one(const LsArgs& A, const LsInst& I, int64_t el, int i)
{
    const int32_t* rp = A.row_ptr + I.rp_off;
    const int32_t* ci = A.col_idx + I.ci_off;
    const int s0 = rp[el], s1 = rp[el + 1];
    const int64_t c0 = (int64_t)s0 - el;
    for (int sl = s0 + 1; sl < s1; ++sl) {
        const double* a = A.A64 + I.val_off + ((int64_t)sl * N + i) * N;
        const double* d = A.Dinv64 + I.dinv_off + (int64_t)ci[sl] * N * N;
        P* out = (P*)A.Ahat + I.ahat_off + ((c0 + (sl - s0 - 1)) * N + i) * N;
        double ar[N];
#pragma unroll
        for (int k = 0; k < N; ++k) ar[k] = a[k];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) s += ar[k] * d[k * N + c];
            out[c] = (P)s;
        }
    }
    const double* dd = A.Dinv64 + I.dinv_off + (el * N + i) * N;
    P* dp = (P*)A.DinvP + I.dinv_off + (el * N + i) * N;
#pragma unroll
    for (int c = 0; c < N; ++c) dp[c] = (P)dd[c];
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_form_kernel(const LsArgs A)
{
    ElemLane e;
    if (!ls_elem_lane(A, e)) return;
    const LsInst& I = A.inst[e.inst];
    if (I.k == 1) ls_form_one<P, 3>(A, I, e.el, e.j);
    else ls_form_one<P, 6>(A, I, e.el, e.j);
}

// ---------------------------------------------------------------------------
// norms, residual, cycle control
// ---------------------------------------------------------------------------
// ||F||^2 per instance: row chunks -> red[inst][chunk]
__global__ __launch_bounds__(LS_BT) void ls_bnorm_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const double* f = A.rhs + I.x_off;
    double acc = 0.0;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) acc += f[t] * f[t];
    acc = ls_block_sum(acc, sh);
    if (threadIdx.x == 0) A.red[I.red_off + ch] = acc;
}

// r = F - A x (FP64); element blocks -> red2[inst][element block]
__global__ __launch_bounds__(LS_BT) void ls_residual_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64];
    ElemLane e;
    const bool act = ls_elem_lane(A, e);
    const LsInst& I = A.inst[e.inst];
    double v = 0.0;
    if (act && A.state[e.inst].active) {
        const int N = e.n;
        const int32_t* rp = A.row_ptr + I.rp_off;
        const int32_t* ci = A.col_idx + I.ci_off;
        const double* x = A.x + I.x_off;
        double s = A.rhs[I.x_off + e.el * N + e.j];
        for (int sl = rp[e.el]; sl < rp[e.el + 1]; ++sl) {
            const double* blk = A.A64 + I.val_off + ((int64_t)sl * N + e.j) * N;
            const double* xv = x + (int64_t)ci[sl] * N;
            for (int c = 0; c < N; ++c) s -= blk[c] * xv[c];
        }
        A.r[I.x_off + e.el * N + e.j] = s;
        v = s * s;
    }
    v = ls_block_sum(v, sh);
    if (threadIdx.x == 0) A.red2[I.red2_off + (blockIdx.x - A.eblk[e.inst])] = v;
}

// one block per instance: ||F|| (first call), true relative residual,
// convergence / cap decisions, report, and the next cycle's state
__global__ __launch_bounds__(LS_BT) void ls_check_kernel(const LsArgs A, int first)
{
    __shared__ double sh[LS_BT / 64];
    const int i = blockIdx.x;
    const LsInst& I = A.inst[i];
    LsState& S = A.state[i];
    if (!S.active) return;
    if (first) {
        double a = 0.0;
        for (int c = threadIdx.x; c < I.nchunks; c += LS_BT) a += A.red[I.red_off + c];
        a = ls_block_sum(a, sh);
        if (threadIdx.x == 0) S.bnorm = sqrt(a);
        __syncthreads();
    }
    double a = 0.0;
    for (int c = threadIdx.x; c < I.neblk; c += LS_BT) a += A.red2[I.red2_off + c];
    a = ls_block_sum(a, sh);
    // the true residual judges the initial guess: one worse than zero is
    // replaced by x = 0, for which r = F
    __shared__ int reject;
    if (threadIdx.x == 0)
        reject = first && S.bnorm > 0.0 && isfinite(S.bnorm) && !(sqrt(a) <= A.guess_limit * S.bnorm);
    __syncthreads();
    if (reject) {
        double* x = A.x + I.x_off;
        double* r = A.r + I.x_off;
        const double* f = A.rhs + I.x_off;
        for (int64_t t = threadIdx.x; t < I.n; t += LS_BT) {
            x[t] = 0.0;
            r[t] = f[t];
        }
    }
    if (threadIdx.x != 0) return;
    dg_solve_report& R = A.reports[I.id];
    if (!first) { S.its += S.J; S.cycles += 1; }
    double beta = sqrt(a);
    if (first) {
        R.guess_rejected = reject;
        R.persistent = 0;
        R.rel_res0 = S.bnorm > 0.0 ? beta / S.bnorm : 0.0;
        if (reject) beta = S.bnorm;
    }
    const double rel = S.bnorm > 0.0 ? beta / S.bnorm : 0.0;
    R.rel_res = rel;
    R.iters = S.its;
    R.cycles = S.cycles;
    R.reorth_passes = 0;
    int st = DG_NOT_CONVERGED;
    bool done = false;
    if (S.status == DG_ERR_NONFINITE || !isfinite(rel) || !isfinite(S.bnorm)) { st = DG_ERR_NONFINITE; done = true; }
    else if (rel <= A.rel_tol) { st = DG_OK; done = true; }
    else if (S.its >= A.max_iters) { st = DG_NOT_CONVERGED; done = true; }
    R.status = st;
    if (done) {
        S.active = 0;
        S.stop = 1;
        return;
    }
    S.beta = beta;
    S.cyctol = fmax(A.mixed ? A.inner_tol * beta : 0.0, A.rel_tol * S.bnorm);
    S.mcyc = min(I.m, A.max_iters - S.its);
    S.J = 0;
    S.stop = 0;
    A.g[I.h_off] = beta;
    atomicAdd(A.counters + 0, 1);  // instances active in this cycle
    atomicAdd(A.counters + 1, 1);  // cycles still running
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_cycle_init_kernel(const LsArgs A)
{
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsInst& I = A.inst[i];
    const LsState& S = A.state[i];
    if (!S.active) return;
    const int64_t ch = b - A.rblk[i];
    const double inv = 1.0 / S.beta;
    P* V = (P*)A.V + I.v_off;
    const double* r = A.r + I.x_off;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) V[t] = (P)(r[t] * inv);
}

// ---------------------------------------------------------------------------
// Arnoldi step kernels
// ---------------------------------------------------------------------------
// w = Ahat v_J, or with second = 1 the two-vector block's w1 = Ahat w
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_spmv_kernel(const LsArgs A, int second)
{
    ElemLane e;
    if (!ls_elem_lane(A, e)) return;
    const LsState& S = A.state[e.inst];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[e.inst];
    const int N = e.n;
    const int32_t* rp = A.row_ptr + I.rp_off;
    const int32_t* ci = A.col_idx + I.ci_off;
    const P* v = second ? (const P*)A.w + I.x_off : (const P*)A.V + I.v_off + (int64_t)S.J * I.n;
    const P* Ah = (const P*)A.Ahat + I.ahat_off;
    const int s0 = rp[e.el], s1 = rp[e.el + 1];
    const int64_t c0 = (int64_t)s0 - e.el;
    double s = (double)v[e.el * N + e.j];
    for (int sl = s0 + 1; sl < s1; ++sl) {
        const P* blk = Ah + ((c0 + (sl - s0 - 1)) * N + e.j) * N;
        const P* xv = v + (int64_t)ci[sl] * N;
        for (int c = 0; c < N; ++c) s += (double)blk[c] * (double)xv[c];
    }
    ((P*)(second ? A.w1 : A.w))[I.x_off + e.el * N + e.j] = (P)s;
}

// partial V_c . w (c <= J) and w . w (c = J+1) over one row chunk
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_multidot_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64][LS_CT];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = S.J, ncols = J + 2;
    const P* V = (const P*)A.V + I.v_off;
    const P* w = (const P*)A.w + I.x_off;
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* part = A.part + I.part_off;
    for (int t0 = 0; t0 < ncols; t0 += LS_CT) {
        const P* col[LS_CT];
#pragma unroll
        for (int c = 0; c < LS_CT; ++c) col[c] = (t0 + c <= J) ? V + (int64_t)(t0 + c) * I.n : w;
        double ac[LS_CT];
#pragma unroll
        for (int c = 0; c < LS_CT; ++c) ac[c] = 0.0;
        for (int64_t t = r0 + threadIdx.x; t < r1; t += LS_BT) {
            const double wv = (double)w[t];
#pragma unroll
            for (int c = 0; c < LS_CT; ++c) ac[c] += (double)col[c][t] * wv;
        }
#pragma unroll
        for (int c = 0; c < LS_CT; ++c) {
            const double v = ls_wave_sum(ac[c]);
            if (lane == 0) sh[wave][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < LS_CT && t0 + (int)threadIdx.x < ncols) {
            const int c = threadIdx.x;
            part[(int64_t)(t0 + c) * I.nchunks + ch] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
        }
        __syncthreads();
    }
}

// one block per instance: h[c] = sum over chunks (J + 2 columns, or 2 (J + 1)
// for a two-vector block)
__global__ __launch_bounds__(LS_BT) void ls_reduce_kernel(const LsArgs A, int block2)
{
    const int i = blockIdx.x;
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const double* part = A.part + I.part_off;
    const int ncols = block2 ? 2 * (S.J + 1) : S.J + 2;
    for (int c = threadIdx.x; c < ncols; c += LS_BT) {
        const double* pc = part + (int64_t)c * I.nchunks;
        double s = 0.0;
        int ch = 0;
        for (; ch + LS_BATCH <= I.nchunks; ch += LS_BATCH) {  // loads issued together, summed in order
            double v[LS_BATCH];
#pragma unroll
            for (int u = 0; u < LS_BATCH; ++u) v[u] = pc[ch + u];
#pragma unroll
            for (int u = 0; u < LS_BATCH; ++u) s += v[u];
        }
        for (; ch < I.nchunks; ++ch) s += pc[ch];
        A.hcol[I.hc_off + c] = s;
    }
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_update_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = S.J;
    const P* V = (const P*)A.V + I.v_off;
    P* w = (P*)A.w + I.x_off;
    const double* h = A.hcol + I.hc_off;
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int64_t n = I.n;
    double acc = 0.0;
    // E rows per thread advance through the columns together (4 columns x E
    // rows of loads in flight)
    constexpr int E = 4;
    for (int64_t t0 = r0 + threadIdx.x; t0 < r1; t0 += (int64_t)LS_BT * E) {
        double wr[E];
        bool in[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t t = t0 + (int64_t)e * LS_BT;
            in[e] = t < r1;
            wr[e] = in[e] ? (double)w[t] : 0.0;
        }
        int c = 0;
        for (; c + 3 <= J; c += 4) {
            const double h0 = h[c], h1 = h[c + 1], h2 = h[c + 2], h3 = h[c + 3];
            const P* v0 = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e])
                    wr[e] -= h0 * (double)v0[t] + h1 * (double)v0[t + n] + h2 * (double)v0[t + 2 * n] +
                             h3 * (double)v0[t + 3 * n];
            }
        }
        for (; c <= J; ++c) {
            const double hc = h[c];
            const P* vc = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e]) wr[e] -= hc * (double)vc[t];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (in[e]) {
                const P pv = (P)wr[e];
                w[t0 + (int64_t)e * LS_BT] = pv;
                acc += (double)pv * (double)pv;
            }
        }
    }
    acc = ls_block_sum(acc, sh);
    if (threadIdx.x == 0) A.red[I.red_off + ch] = acc;
}

// one block of 64 threads per instance
__global__ __launch_bounds__(64) void ls_givens_kernel(const LsArgs A)
{
    const int i = blockIdx.x;
    LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    __shared__ double sc[LS_GV], ss[LS_GV], sh2[LS_GV + 1], so[LS_GV];
    __shared__ double carry, wn;
    const int j = S.J;
    const int ldh = I.m + 1;
    double* H = A.H + I.H_off;
    double* cs = A.cs + I.h_off;
    double* sn = A.sn + I.h_off;
    double* g = A.g + I.h_off;
    const double* hcol = A.hcol + I.hc_off;
    double a = 0.0;
    for (int c = threadIdx.x; c < I.nchunks; c += 64) a += A.red[I.red_off + c];
    a = ls_wave_sum(a);
    if (threadIdx.x == 0) { wn = a; carry = hcol[0]; }
    __syncthreads();
    double* col = H + (int64_t)j * ldh;
    for (int i0 = 0; i0 < j; i0 += LS_GV) {
        const int cnt = min(j - i0, LS_GV);
        for (int t = threadIdx.x; t < cnt; t += 64) {
            sc[t] = cs[i0 + t];
            ss[t] = sn[i0 + t];
            sh2[t + 1] = hcol[i0 + t + 1];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double av = carry;
            for (int t = 0; t < cnt; ++t) {
                const double bv = sh2[t + 1];
                so[t] = sc[t] * av + ss[t] * bv;
                av = -ss[t] * av + sc[t] * bv;
            }
            carry = av;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 64) col[i0 + t] = so[t];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double hn = sqrt(wn);
    const double av = carry;
    const double d = sqrt(av * av + hn * hn);
    cs[j] = d == 0.0 ? 1.0 : av / d;
    sn[j] = d == 0.0 ? 0.0 : hn / d;
    col[j] = d;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    S.J = j + 1;
    const bool brk = !(hn > 1e-300) || !isfinite(hn);
    S.invh = brk ? 0.0 : 1.0 / hn;
    if (fabs(g[j + 1]) <= S.cyctol || brk || j + 1 >= S.mcyc) {
        S.stop = 1;
        atomicSub(A.counters + 1, 1);
    }
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_normalize_kernel(const LsArgs A)
{
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const P sc = (P)S.invh;
    P* vn = (P*)A.V + I.v_off + (int64_t)S.J * I.n;
    const P* w = (const P*)A.w + I.x_off;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) vn[t] = w[t] * sc;
}

// ---------------------------------------------------------------------------
// Two-vector blocks (as in the single-system solver): w0 = Ahat v_J and
// w1 = Ahat w0 are projected against v_0..v_J in one pass over the basis and
// updated in a second, the 2 x 2 Gram matrix of the results is factored by
// Cholesky, and the two Hessenberg columns follow from the block relations.
// ---------------------------------------------------------------------------
constexpr int LS_CT2 = 8;  // columns per tile with two right-hand sides

// partial V_c . w_r (c <= J, r = 0, 1) over one row chunk, at part[(r (J+1) + c) nchunks + chunk]
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_multidot2_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64][2 * LS_CT2];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = S.J, ncols = J + 1;
    const P* V = (const P*)A.V + I.v_off;
    const P* w0 = (const P*)A.w + I.x_off;
    const P* w1 = (const P*)A.w1 + I.x_off;
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* part = A.part + I.part_off;
    for (int t0 = 0; t0 < ncols; t0 += LS_CT2) {
        const P* col[LS_CT2];
#pragma unroll
        for (int c = 0; c < LS_CT2; ++c) col[c] = (t0 + c <= J) ? V + (int64_t)(t0 + c) * I.n : w0;  // past J: discarded
        double a0[LS_CT2], a1[LS_CT2];
#pragma unroll
        for (int c = 0; c < LS_CT2; ++c) a0[c] = a1[c] = 0.0;
        for (int64_t t = r0 + threadIdx.x; t < r1; t += LS_BT) {
            const double x0 = (double)w0[t], x1 = (double)w1[t];
#pragma unroll
            for (int c = 0; c < LS_CT2; ++c) {
                const double v = (double)__builtin_nontemporal_load(col[c] + t);  // streamed
                a0[c] += v * x0;
                a1[c] += v * x1;
            }
        }
#pragma unroll
        for (int c = 0; c < LS_CT2; ++c) {
            const double v0 = ls_wave_sum(a0[c]), v1 = ls_wave_sum(a1[c]);
            if (lane == 0) {
                sh[wave][c] = v0;
                sh[wave][LS_CT2 + c] = v1;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * LS_CT2) {
            const int rr = threadIdx.x / LS_CT2, c = threadIdx.x - rr * LS_CT2;
            if (t0 + c < ncols)
                part[((int64_t)rr * ncols + t0 + c) * I.nchunks + ch] =
                    (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
        }
        __syncthreads();
    }
}

// w_r -= sum_{c<=J} R_r[c] V_c (R_0 = hcol[0..J], R_1 = hcol[J+1..2J+1]) and the
// Gram partials u0.u0, u0.u1, u1.u1 at red[red_off + k nchunks + chunk]
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_update2_kernel(const LsArgs A)
{
    __shared__ double sh[LS_BT / 64];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = S.J;
    const P* V = (const P*)A.V + I.v_off;
    P* w0 = (P*)A.w + I.x_off;
    P* w1 = (P*)A.w1 + I.x_off;
    const double* R0 = A.hcol + I.hc_off;
    const double* R1 = R0 + (J + 1);
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int64_t n = I.n;
    double g00 = 0.0, g01 = 0.0, g11 = 0.0;
    constexpr int E = 4;
    for (int64_t t0 = r0 + threadIdx.x; t0 < r1; t0 += (int64_t)LS_BT * E) {
        double u0[E], u1[E];
        bool in[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t t = t0 + (int64_t)e * LS_BT;
            in[e] = t < r1;
            u0[e] = in[e] ? (double)w0[t] : 0.0;
            u1[e] = in[e] ? (double)w1[t] : 0.0;
        }
        int c = 0;
        for (; c + 3 <= J; c += 4) {
            const double p0 = R0[c], p1 = R0[c + 1], p2 = R0[c + 2], p3 = R0[c + 3];
            const double q0 = R1[c], q1 = R1[c + 1], q2 = R1[c + 2], q3 = R1[c + 3];
            const P* v0 = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e]) {
                    const double a = (double)__builtin_nontemporal_load(v0 + t),  // streamed
                                 bb = (double)__builtin_nontemporal_load(v0 + t + n),
                                 cc = (double)__builtin_nontemporal_load(v0 + t + 2 * n),
                                 d = (double)__builtin_nontemporal_load(v0 + t + 3 * n);
                    u0[e] -= p0 * a + p1 * bb + p2 * cc + p3 * d;
                    u1[e] -= q0 * a + q1 * bb + q2 * cc + q3 * d;
                }
            }
        }
        for (; c <= J; ++c) {
            const double p0 = R0[c], q0 = R1[c];
            const P* vc = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e]) {
                    const double a = (double)__builtin_nontemporal_load(vc + t);
                    u0[e] -= p0 * a;
                    u1[e] -= q0 * a;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (in[e]) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                const P a = (P)u0[e], bb = (P)u1[e];
                w0[t] = a;
                w1[t] = bb;
                g00 += (double)a * (double)a;
                g01 += (double)a * (double)bb;
                g11 += (double)bb * (double)bb;
            }
        }
    }
    g00 = ls_block_sum(g00, sh);
    g01 = ls_block_sum(g01, sh);
    g11 = ls_block_sum(g11, sh);
    if (threadIdx.x == 0) {
        double* red = A.red + I.red_off;
        red[ch] = g00;
        red[I.nchunks + ch] = g01;
        red[2 * I.nchunks + ch] = g11;
    }
}

// previous Givens rotations applied to colv[0..count] in LDS (thread 0 runs the
// chain; the rotations are staged in chunks by the 64 threads)
// Rotations 0..count-1 applied to col0 and, when ncol = 2, col1: lane l takes
// column l, the LDS loads of LS_BATCH steps issued together
__device__ void ls_rotate(double* col0, double* col1, int ncol, int count, const double* __restrict__ cs,
                          const double* __restrict__ sn, double* sc, double* ss)
{
    const int l = threadIdx.x;
    double* colv = l == 0 ? col0 : col1;
    __syncthreads();
    double a = l < ncol ? colv[0] : 0.0;
    for (int i0 = 0; i0 < count; i0 += LS_GV) {
        const int cnt = min(count - i0, LS_GV);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 64) {
            sc[t] = cs[i0 + t];
            ss[t] = sn[i0 + t];
        }
        __syncthreads();
        if (l < ncol) {
            double* cv = colv + i0;
            int t = 0;
            for (; t + LS_BATCH <= cnt; t += LS_BATCH) {
                double c[LS_BATCH], s[LS_BATCH], b[LS_BATCH], o[LS_BATCH];
#pragma unroll
                for (int u = 0; u < LS_BATCH; ++u) {
                    c[u] = sc[t + u];
                    s[u] = ss[t + u];
                    b[u] = cv[t + u + 1];  // not yet written: this batch writes cv[t .. t + LS_BATCH - 1]
                }
#pragma unroll
                for (int u = 0; u < LS_BATCH; ++u) {
                    o[u] = c[u] * a + s[u] * b[u];
                    a = -s[u] * a + c[u] * b[u];
                }
#pragma unroll
                for (int u = 0; u < LS_BATCH; ++u) cv[t + u] = o[u];
            }
            for (; t < cnt; ++t) {
                const double bv = cv[t + 1];
                cv[t] = sc[t] * a + ss[t] * bv;
                a = -ss[t] * a + sc[t] * bv;
            }
        }
    }
    if (l < ncol) colv[count] = a;
    __syncthreads();
}

// one block of 64 threads per instance: Gram sums, Cholesky, the two raw
// Hessenberg columns (Hr, leading dimension m + 2) and, rotated, into H;
// residual estimates and stop tests.  Dynamic LDS: two columns of max_m + 4.
__global__ __launch_bounds__(64) void ls_block_givens_kernel(const LsArgs A, int step)
{
    extern __shared__ double dyn[];
    __shared__ double sc[LS_GV], ss[LS_GV];
    __shared__ double fac[3];
    __shared__ int flags[2];  // take the second column, stop after the first
    const int i = blockIdx.x;
    LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const int j = S.J, mcyc = S.mcyc, ldh = I.m + 1, ldr = I.m + 2;
    double* colA = dyn;
    double* colB = dyn + (I.m + 4);
    double* H = A.H + I.H_off;
    double* Hr = A.Hr + I.Hr_off;
    double* cs = A.cs + I.h_off;
    double* sn = A.sn + I.h_off;
    double* g = A.g + I.h_off;
    const double* R0 = A.hcol + I.hc_off;
    const double* R1 = R0 + (j + 1);
    const double* red = A.red + I.red_off;
    double a00 = 0.0, a01 = 0.0, a11 = 0.0;
    for (int c = threadIdx.x; c < I.nchunks; c += 64) {
        a00 += red[c];
        a01 += red[I.nchunks + c];
        a11 += red[2 * I.nchunks + c];
    }
    a00 = ls_wave_sum(a00);
    a01 = ls_wave_sum(a01);
    a11 = ls_wave_sum(a11);
    for (int t = threadIdx.x; t <= j; t += 64) colA[t] = R0[t];
    if (threadIdx.x == 0) {
        const double r11 = sqrt(a00);
        const bool brk1 = !(r11 > 1e-300) || !isfinite(r11);
        const double r12 = brk1 ? 0.0 : a01 / r11;
        const double d = a11 - r12 * r12;
        const double r22 = d > 0.0 ? sqrt(d) : 0.0;
        const bool ok2 = !brk1 && isfinite(r22) && r22 > 1e-8 * sqrt(a11);
        fac[0] = r11;
        fac[1] = r12;
        fac[2] = r22;
        colA[j + 1] = r11;
        S.q1 = brk1 ? 0.0 : 1.0 / r11;
        S.q2a = ok2 ? 1.0 / r22 : 0.0;
        S.q2b = ok2 ? -r12 / (r11 * r22) : 0.0;
        flags[0] = ok2 ? 1 : 0;
        flags[1] = brk1 ? 1 : 0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j + 1; t += 64) Hr[t + (int64_t)j * ldr] = colA[t];
    __syncthreads();
    const bool want2 = !flags[1] && j + 1 < mcyc;
    if (want2) {
        const double r11 = fac[0];
        for (int t = threadIdx.x; t <= j + 1; t += 64) {
            double acc = 0.0;
            int c = t > 0 ? t - 1 : 0;
            for (; c + LS_BATCH <= j + 1; c += LS_BATCH) {  // loads issued together, summed in order
                double h[LS_BATCH], r[LS_BATCH];
#pragma unroll
                for (int u = 0; u < LS_BATCH; ++u) {
                    h[u] = Hr[t + (int64_t)(c + u) * ldr];
                    r[u] = R0[c + u];
                }
#pragma unroll
                for (int u = 0; u < LS_BATCH; ++u) acc += h[u] * r[u];
            }
            for (; c <= j; ++c) acc += Hr[t + (int64_t)c * ldr] * R0[c];
            colB[t] = ((t <= j ? R1[t] : fac[1]) - acc) / r11;
        }
        if (threadIdx.x == 0) colB[j + 2] = fac[2] / r11;
        __syncthreads();
        for (int t = threadIdx.x; t <= j + 2; t += 64) Hr[t + (int64_t)(j + 1) * ldr] = colB[t];
    }
    ls_rotate(colA, colB, want2 ? 2 : 1, j, cs, sn, sc, ss);  // earlier blocks' rotations on both columns
    if (threadIdx.x == 0) {
        const double a = colA[j], bv = colA[j + 1];
        const double d = sqrt(a * a + bv * bv);
        cs[j] = d == 0.0 ? 1.0 : a / d;
        sn[j] = d == 0.0 ? 0.0 : bv / d;
        colA[j] = d;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        if (flags[1] || fabs(g[j + 1]) <= S.cyctol || j + 1 >= mcyc || !want2) flags[1] = 1;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j; t += 64) H[t + (int64_t)j * ldh] = colA[t];
    if (flags[1]) {
        if (threadIdx.x == 0) {
            S.jb = j;
            S.bstep = step;
            S.J = j + 1;
            S.stop = 1;
            atomicSub(A.counters + 1, 1);
        }
        return;
    }
    if (threadIdx.x == 0) {
        const int k = j + 1;
        {  // the first column's rotation on the second
            const double a = colB[j], bv = colB[k];
            colB[j] = cs[j] * a + sn[j] * bv;
            colB[k] = -sn[j] * a + cs[j] * bv;
        }
        const double a = colB[k], bv = colB[k + 1];
        const double d = sqrt(a * a + bv * bv);
        cs[k] = d == 0.0 ? 1.0 : a / d;
        sn[k] = d == 0.0 ? 0.0 : bv / d;
        colB[k] = d;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        S.jb = j;
        S.bstep = step;
        S.J = k + 1;
        if (!flags[0] || fabs(g[k + 1]) <= S.cyctol || k + 1 >= mcyc) {
            S.stop = 1;
            atomicSub(A.counters + 1, 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j + 1; t += 64) H[t + (int64_t)(j + 1) * ldh] = colB[t];
}

// v_{jb+1} = q1 u0 and, unless the cycle stopped, v_{jb+2} = q2a u1 + q2b u0,
// for instances whose block of this step took both columns
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_normalize2_kernel(const LsArgs A, int step)
{
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!S.active || S.bstep != step || S.J != S.jb + 2) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const bool second = !S.stop;
    const double a = S.q1, qa = S.q2a, qb = S.q2b;
    P* o1 = (P*)A.V + I.v_off + (int64_t)(S.jb + 1) * I.n;
    P* o2 = o1 + I.n;
    const P* w0 = (const P*)A.w + I.x_off;
    const P* w1 = (const P*)A.w1 + I.x_off;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) {
        const double u0 = (double)w0[t];
        o1[t] = (P)(u0 * a);
        if (second) o2[t] = (P)((double)w1[t] * qa + u0 * qb);
    }
}

// ---------------------------------------------------------------------------
// end of a cycle: y = R^{-1} g, u = V y, x += D^{-1} u
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LS_BT) void ls_trisolve_kernel(const LsArgs A)
{
    const int i = blockIdx.x;
    const LsState& S = A.state[i];
    if (!S.active) return;
    const LsInst& I = A.inst[i];
    const int J = S.J;
    const int ldh = I.m + 1;
    const double* H = A.H + I.H_off;
    double* g = A.g + I.h_off;
    double* y = A.y + I.h_off;
    __shared__ double yi_s;
    for (int r = J - 1; r >= 0; --r) {
        if (threadIdx.x == 0) {
            yi_s = g[r] / H[r + (int64_t)r * ldh];
            y[r] = yi_s;
        }
        __syncthreads();
        const double yi = yi_s;
        for (int k = threadIdx.x; k < r; k += LS_BT) g[k] -= H[k + (int64_t)r * ldh] * yi;
        __syncthreads();
    }
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_combine_kernel(const LsArgs A)
{
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& S = A.state[i];
    if (!S.active) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const P* V = (const P*)A.V + I.v_off;
    const double* y = A.y + I.h_off;
    P* u = (P*)A.w + I.x_off;  // w is free at the end of a cycle
    const int J = S.J;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) {
        double s = 0.0;
        for (int c = 0; c < J; ++c) s += y[c] * (double)V[(int64_t)c * I.n + t];
        u[t] = (P)s;
    }
}

template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_dinv_update_kernel(const LsArgs A)
{
    ElemLane e;
    if (!ls_elem_lane(A, e)) return;
    if (!A.state[e.inst].active) return;
    const LsInst& I = A.inst[e.inst];
    const int N = e.n;
    const P* d = (const P*)A.DinvP + I.dinv_off + (e.el * N + e.j) * N;
    const P* u = (const P*)A.w + I.x_off + e.el * N;
    double s = 0.0;
    for (int c = 0; c < N; ++c) s += (double)d[c] * (double)u[c];
    A.x[I.x_off + e.el * N + e.j] += s;
}

__global__ void ls_zero_counters(int* c) { c[0] = 0; c[1] = 0; }

__global__ void ls_init_kernel(LsState* st, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    LsState s{};
    s.active = 1;
    s.stop = 1;
    st[i] = s;
}

int ls_init(const LsArgs& A, hipStream_t st)
{
    if (A.count <= 0) return DG_OK;
    hipLaunchKernelGGL(ls_init_kernel, dim3((A.count + 255) / 256), dim3(256), 0, st, A.state, A.count);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
template <typename P>
static int ls_solve_p(const LsArgs& A, int64_t n_eblk, int64_t n_rblk, int max_m, hipStream_t st, dg_progress_fn fn,
                      void* user, int done_before, int total)
{
    const dim3 be(LS_BT), ge((unsigned)n_eblk), gr((unsigned)n_rblk), gi((unsigned)A.count);
    hipLaunchKernelGGL(ls_invert_kernel, ge, be, 0, st, A);
    hipLaunchKernelGGL((ls_form_kernel<P>), ge, be, 0, st, A);
    hipLaunchKernelGGL(ls_bnorm_kernel, gr, be, 0, st, A);
    int first = 1;
    int h[2];
    int step = 1;  // host step index of the two-vector blocks, unique over the whole solve
    for (;;) {
        hipLaunchKernelGGL(ls_zero_counters, dim3(1), dim3(1), 0, st, A.counters);
        hipLaunchKernelGGL(ls_residual_kernel, ge, be, 0, st, A);
        hipLaunchKernelGGL(ls_check_kernel, gi, be, 0, st, A, first);
        first = 0;
        DG_HIP_CHECK(hipMemcpyAsync(h, A.counters, sizeof(h), hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipStreamSynchronize(st));
        if (fn) fn(user, done_before + (A.count - h[0]), total);
        if (h[0] == 0) break;
        hipLaunchKernelGGL((ls_cycle_init_kernel<P>), gr, be, 0, st, A);
        const size_t dyn = sizeof(double) * 2 * (size_t)(max_m + 4);
        for (int j = 0; A.block == 2 && j < max_m; j += 2, ++step) {
            hipLaunchKernelGGL((ls_spmv_kernel<P>), ge, be, 0, st, A, 0);
            hipLaunchKernelGGL((ls_spmv_kernel<P>), ge, be, 0, st, A, 1);
            hipLaunchKernelGGL((ls_multidot2_kernel<P>), gr, be, 0, st, A);
            hipLaunchKernelGGL(ls_reduce_kernel, gi, be, 0, st, A, 1);
            hipLaunchKernelGGL((ls_update2_kernel<P>), gr, be, 0, st, A);
            hipLaunchKernelGGL(ls_block_givens_kernel, gi, dim3(64), dyn, st, A, step);
            hipLaunchKernelGGL((ls_normalize2_kernel<P>), gr, be, 0, st, A, step);
            if ((j & 7) == 6) {  // every 8 steps: stop early once every cycle has ended
                DG_HIP_CHECK(hipMemcpyAsync(h, A.counters, sizeof(h), hipMemcpyDeviceToHost, st));
                DG_HIP_CHECK(hipStreamSynchronize(st));
                if (h[1] <= 0) break;
            }
        }
        for (int j = 0; A.block != 2 && j < max_m; ++j) {
            hipLaunchKernelGGL((ls_spmv_kernel<P>), ge, be, 0, st, A, 0);
            hipLaunchKernelGGL((ls_multidot_kernel<P>), gr, be, 0, st, A);
            hipLaunchKernelGGL(ls_reduce_kernel, gi, be, 0, st, A, 0);
            hipLaunchKernelGGL((ls_update_kernel<P>), gr, be, 0, st, A);
            hipLaunchKernelGGL(ls_givens_kernel, gi, dim3(64), 0, st, A);
            hipLaunchKernelGGL((ls_normalize_kernel<P>), gr, be, 0, st, A);
            if ((j & 7) == 7) {  // every 8 steps: stop early once every cycle has ended
                DG_HIP_CHECK(hipMemcpyAsync(h, A.counters, sizeof(h), hipMemcpyDeviceToHost, st));
                DG_HIP_CHECK(hipStreamSynchronize(st));
                if (h[1] <= 0) break;
            }
        }
        hipLaunchKernelGGL(ls_trisolve_kernel, gi, be, 0, st, A);
        hipLaunchKernelGGL((ls_combine_kernel<P>), gr, be, 0, st, A);
        hipLaunchKernelGGL((ls_dinv_update_kernel<P>), ge, be, 0, st, A);
        DG_HIP_CHECK(hipGetLastError());
    }
    return DG_OK;
}

int ls_solve(const LsArgs& A, int64_t n_eblk, int64_t n_rblk, int max_m, int mixed, hipStream_t st,
             dg_progress_fn fn, void* user, int done_before, int total)
{
    if (A.count <= 0) return DG_OK;
    return mixed ? ls_solve_p<float>(A, n_eblk, n_rblk, max_m, st, fn, user, done_before, total)
                 : ls_solve_p<double>(A, n_eblk, n_rblk, max_m, st, fn, user, done_before, total);
}

int64_t ls_elem_blocks(int k, int64_t T)
{
    const int n = (k + 1) * (k + 2) / 2, epw = 64 / n;
    const int64_t per = (int64_t)(LS_BT / 64) * epw;
    return (T + per - 1) / per;
}

int64_t ls_row_chunks(int64_t n) { return (n + LS_CH - 1) / LS_CH; }

}  // namespace dg
