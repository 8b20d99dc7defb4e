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
#include "mfma.h"

namespace dg {

constexpr int LS_BT = 256;       // threads per block
constexpr int LS_CH = 1024;      // rows per row chunk (one workgroup each); measured fastest of 512..16384
constexpr int LS_CT = 16;        // Gram-Schmidt columns reduced together (8: same, 32: slower)
constexpr int LS_GV = 512;       // Givens staging chunk
constexpr int LS_BATCH = 8;      // loads issued together in the serial loops of the block kernels
constexpr int LS_GT = 512;       // threads of the block Givens kernel (its Hessenberg products take a row per
constexpr int LS_SEG = 4;        // group of LS_SEG lanes)

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
// every cycle of the chunk has ended (counters[1] counts the running ones; it
// only falls while a cycle's Arnoldi blocks run): the launches of the rest of
// the cycle have nothing to do.  Only kernels that run before the block's
// Givens kernel may use it, since that kernel takes the count to zero.
__device__ __forceinline__ bool ls_all_ended(const LsArgs& A) { return A.counters[1] <= 0; }

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
// Row j of element el of Ahat v for blocks of N <= 6: a triangle has at most
// three neighbours, and the loads of all three are issued before the first
// product (absent ones read the row `own`, which always exists, and are not
// added); the sums keep the neighbour order.
template <typename P, int N>
__device__ __forceinline__ double ls_spmv_row(const P* Ah, const int32_t* rp, const int32_t* ci, const P* v,
                                              const P* own, int64_t el, int j, double cid)
{
    const int s0 = rp[el], s1 = rp[el + 1];
    const int64_t c0 = (int64_t)s0 - el;
    double s = cid * (double)v[el * N + j];  // cid = 1 - theta: the identity blocks of Ahat - theta I
    constexpr int NB = 3;
    const int nb = s1 - s0 - 1;
    P bl[NB][N], xx[NB][N];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const bool has = q < nb;
        const P* blk = has ? Ah + ((c0 + q) * N + j) * N : own;
        const P* xv = has ? v + (int64_t)ci[s0 + 1 + q] * N : v + el * N;
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
            for (int c = 0; c < N; ++c) s += (double)bl[q][c] * (double)xx[q][c];
        }
    for (int sl = s0 + 1 + NB; sl < s1; ++sl) {  // not reached on triangle meshes
        const P* blk = Ah + ((c0 + (sl - s0 - 1)) * N + j) * N;
        const P* xv = v + (int64_t)ci[sl] * N;
#pragma unroll
        for (int c = 0; c < N; ++c) s += (double)blk[c] * (double)xv[c];
    }
    return s;
}

// vector r of an Arnoldi block (w, w1, w2, then wx)
template <typename P>
__device__ __forceinline__ P* ls_block_vec(const LsArgs& A, int r)
{
    return (P*)(r == 0 ? A.w : r == 1 ? A.w1 : r == 2 ? A.w2 : A.wx[r - 3]);
}

template <typename P>
// Workgroups stay in the hardware's round-robin order over the XCDs: dealing each XCD a contiguous eighth of the
// batch's element blocks (as the single-system SpMV does) was slower here (256-instance sample: 37.2 -> 47.5 us
// per FP64 launch), the instances that had finished their cycle leaving whole XCDs idle.
__global__ __launch_bounds__(LS_BT) void ls_spmv_kernel(const LsArgs A, int src, double cid)
{
    if (ls_all_ended(A)) return;
    ElemLane e;
    if (!ls_elem_lane(A, e)) return;
    const LsState& S = A.state[e.inst];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[e.inst];
    const int N = e.n;
    const int32_t* rp = A.row_ptr + I.rp_off;
    const int32_t* ci = A.col_idx + I.ci_off;
    // src 0: (Ahat - theta I) v_J into w; src r > 0: a block's w_r = (Ahat - theta I) w_{r-1}
    const P* v = src == 0 ? (const P*)A.V + I.v_off + (int64_t)S.J * I.vs : ls_block_vec<P>(A, src - 1) + I.x_off;
    const P* Ah = (const P*)A.Ahat + I.ahat_off;
    const P* own = (const P*)A.DinvP + I.dinv_off + (e.el * N + e.j) * N;  // a row that always exists
    double s;
    switch (N) {  // uniform over the workgroup: one instance per element block
    case 1: s = ls_spmv_row<P, 1>(Ah, rp, ci, v, own, e.el, e.j, cid); break;
    case 3: s = ls_spmv_row<P, 3>(Ah, rp, ci, v, own, e.el, e.j, cid); break;
    case 6: s = ls_spmv_row<P, 6>(Ah, rp, ci, v, own, e.el, e.j, cid); break;
    default: {
        const int s0 = rp[e.el], s1 = rp[e.el + 1];
        const int64_t c0 = (int64_t)s0 - e.el;
        s = cid * (double)v[e.el * N + e.j];
        for (int sl = s0 + 1; sl < s1; ++sl) {
            const P* blk = Ah + ((c0 + (sl - s0 - 1)) * N + e.j) * N;
            const P* xv = v + (int64_t)ci[sl] * N;
            for (int c = 0; c < N; ++c) s += (double)blk[c] * (double)xv[c];
        }
    }
    }
    ls_block_vec<P>(A, src)[I.x_off + e.el * N + e.j] = (P)s;
}

// partial V_c . w (c <= J) and w . w (c = J+1) over one row chunk
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_multidot_kernel(const LsArgs A)
{
    if (ls_all_ended(A)) return;
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
        for (int c = 0; c < LS_CT; ++c) col[c] = (t0 + c <= J) ? V + (int64_t)(t0 + c) * I.vs : w;
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
__global__ __launch_bounds__(LS_BT) void ls_reduce_kernel(const LsArgs A, int nrhs)
{
    const int i = blockIdx.x;
    const LsState& S = A.state[i];
    if (!ls_running(S)) return;
    const LsInst& I = A.inst[i];
    const double* part = A.part + I.part_off;
    const int ncols = nrhs ? nrhs * (S.J + 1) : S.J + 2;  // a block's S (J + 1) dots, or one step's J + 2
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
    if (ls_all_ended(A)) return;
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
    const int64_t n = I.vs;  // basis column stride
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
    P* vn = (P*)A.V + I.v_off + (int64_t)S.J * I.vs;
    const P* w = (const P*)A.w + I.x_off;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) vn[t] = w[t] * sc;
}

// ---------------------------------------------------------------------------
// Arnoldi blocks of S = 2, 3, 6 or 8 vectors (as in the single-system solver):
// w_0 = (Ahat - theta I) v_J and w_i = (Ahat - theta I) w_{i-1} (theta 0 or 1)
// are projected against v_0..v_J in one pass over the basis and updated in a
// second, the S x S Gram matrix of the results is factored by Cholesky, and
// the S Hessenberg columns follow from the block relations W = V R + Q C.
// ---------------------------------------------------------------------------
// columns per tile of the block dot kernel: S x columns accumulators per
// thread, at most 48 (the butterfly sum keeps them in registers)
constexpr int ls_ct2(int S) { return S == 8 ? 6 : 8; }

// Sums NV per-lane values over the 64 lanes of a wave: while the count is even
// each exchange step keeps half of them (the half picked by the step's lane
// bit) and adds the partner's copy of that half, so the work halves per step;
// the rest are summed over the remaining lane bits.  On return lanes with
// (lane & full) == 0 hold the totals of values base .. base + n - 1 in a[0..n).
template <int NV>
__device__ __forceinline__ void ls_butterfly_sum(double (&a)[NV], int lane, int& base, int& n, int& full)
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


// partial V_c . w_r (c <= J, r < S) over one row chunk, at part[(r (J+1) + c) nchunks + chunk]
template <typename P, int S>
__global__ __launch_bounds__(LS_BT) void ls_multidot_block_kernel(const LsArgs A)
{
    if (ls_all_ended(A)) return;
    constexpr int LS_CT2 = ls_ct2(S);
    __shared__ double sh[LS_BT / 64][S * LS_CT2];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& St = A.state[i];
    if (!ls_running(St)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = St.J, ncols = J + 1;
    const P* V = (const P*)A.V + I.v_off;
    const P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = ls_block_vec<P>(A, q) + I.x_off;
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* part = A.part + I.part_off;
    for (int t0 = 0; t0 < ncols; t0 += LS_CT2) {
        const P* col[LS_CT2];
#pragma unroll
        for (int c = 0; c < LS_CT2; ++c) col[c] = (t0 + c <= J) ? V + (int64_t)(t0 + c) * I.vs : wv[0];  // past J: discarded
        double a[S][LS_CT2];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int c = 0; c < LS_CT2; ++c) a[q][c] = 0.0;
        for (int64_t t = r0 + threadIdx.x; t < r1; t += LS_BT) {
            double x[S];
#pragma unroll
            for (int q = 0; q < S; ++q) x[q] = (double)wv[q][t];
#pragma unroll
            for (int c = 0; c < LS_CT2; ++c) {
                const double v = (double)__builtin_nontemporal_load(col[c] + t);  // streamed
#pragma unroll
                for (int q = 0; q < S; ++q) a[q][c] += v * x[q];
            }
        }
        double flat[S * LS_CT2];
#pragma unroll
        for (int q = 0; q < S; ++q)
#pragma unroll
            for (int c = 0; c < LS_CT2; ++c) flat[q * LS_CT2 + c] = a[q][c];
        int base, nv, full;
        ls_butterfly_sum<S * LS_CT2>(flat, lane, base, nv, full);
        if ((lane & full) == 0) {
#pragma unroll
            for (int k = 0; k < S * LS_CT2; ++k)
                if (k < nv) sh[wave][base + k] = flat[k];
        }
        __syncthreads();
        if (threadIdx.x < S * LS_CT2) {
            const int rr = threadIdx.x / LS_CT2, c = threadIdx.x - rr * LS_CT2;
            if (t0 + c < ncols)
                part[((int64_t)rr * ncols + t0 + c) * I.nchunks + ch] =
                    (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
        }
        __syncthreads();
    }
}

// The same partials for blocks of eight vectors on the matrix cores, as the
// single-system solver forms them: for each tile of LS_MF_CT = 32 basis
// columns the chunk's four waves each take a quarter of its rows in 32-row
// pieces, staged in LDS with coalesced loads (the next piece's loads in flight
// during the products), and accumulate V_tile^T W in FP64 16 x 16 x 4 products
// (FP32 data converted; the eight vectors fill half of the 16 product
// columns); the four waves' sums are added in LDS at the end of each tile.
constexpr int LS_MF_CT = 32, LS_MF_CH = 32;
template <typename P>
__global__ __launch_bounds__(LS_BT) void ls_multidot_mfma_kernel(const LsArgs A)
{
    if (ls_all_ended(A)) return;
    constexpr int S = 8, CT = LS_MF_CT, CH = LS_MF_CH, WPB = LS_BT / 64, NA = CT / 16;
    constexpr int STR = sizeof(P) == 8 ? CH + 1 : CH + 2;  // padded row stride of the staged pieces
    constexpr int NSUB = LS_CH / WPB / CH;                  // pieces per wave and tile
    static_assert(NSUB * CH * WPB == LS_CH && CH == 32, "a lane loads row lane % 32 of two columns");
    using Op = MfmaOp<double>;
    using VR = typename Op::V;
    __shared__ P sv[WPB][CT * STR];
    __shared__ P sw[WPB][S * STR];
    __shared__ double red[WPB][CT * S];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& St = A.state[i];
    if (!ls_running(St)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = St.J, ncols = J + 1;
    const int ntiles = (ncols + CT - 1) / CT;
    const P* V = (const P*)A.V + I.v_off;
    const P* wv[S];
#pragma unroll
    for (int v = 0; v < S; ++v) wv[v] = ls_block_vec<P>(A, v) + I.x_off;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, li = lane & 15;
    const int lr = lane & 31, lc = lane >> 5;  // loads: row lr of columns 2 c + lc
    const int64_t wr0 = ch * LS_CH + (int64_t)wave * (NSUB * CH);
    P* mv = sv[wave];
    P* mw = sw[wave];
    double* part = A.part + I.part_off;
    P x[CT / 2], y[S / 2];
    auto load = [&](int s) {
        const int t0 = (s / NSUB) * CT;
        const int64_t r = wr0 + (int64_t)(s % NSUB) * CH + lr;
        const bool in = r < r1;
#pragma unroll
        for (int c = 0; c < CT / 2; ++c) {  // columns past J read column J and are discarded
            const int cc = t0 + 2 * c + lc;
            x[c] = in ? __builtin_nontemporal_load(V + (int64_t)(cc < ncols ? cc : J) * I.vs + r) : P(0);
        }
#pragma unroll
        for (int v = 0; v < S / 2; ++v) y[v] = in ? wv[2 * v + lc][r] : P(0);
    };
    VR acc[NA];
#pragma unroll
    for (int h = 0; h < NA; ++h) acc[h] = VR{0, 0, 0, 0};
    const int total = ntiles * NSUB;
    load(0);
    for (int s = 0; s < total; ++s) {
#pragma unroll
        for (int c = 0; c < CT / 2; ++c) mv[(2 * c + lc) * STR + lr] = x[c];
#pragma unroll
        for (int v = 0; v < S / 2; ++v) mw[(2 * v + lc) * STR + lr] = y[v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (s + 1 < total) load(s + 1);
#pragma unroll
        for (int t = 0; t < CH / 4; ++t) {
            const double bv = (double)mw[(li & 7) * STR + 4 * t + q];
#pragma unroll
            for (int h = 0; h < NA; ++h) {
                const double av = (double)mv[(16 * h + li) * STR + 4 * t + q];
                acc[h] = Op::mac(av, li < S ? bv : 0.0, acc[h]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (s % NSUB == NSUB - 1) {  // end of a tile: the four waves' sums
            const int t0 = (s / NSUB) * CT;
            if (li < S) {
#pragma unroll
                for (int h = 0; h < NA; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v) red[wave][(16 * h + Op::row(q, v)) * S + li] = acc[h][v];
            }
#pragma unroll
            for (int h = 0; h < NA; ++h) acc[h] = VR{0, 0, 0, 0};
            __syncthreads();
            for (int k = threadIdx.x; k < CT * S; k += LS_BT) {
                const int c = k / S, v = k - c * S;
                if (t0 + c < ncols)
                    part[((int64_t)v * ncols + t0 + c) * I.nchunks + ch] =
                        (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
            }
            __syncthreads();
        }
    }
}

// w_r -= sum_{c<=J} R_r[c] V_c (R_r = hcol + r (J+1)) and the Gram partials of
// the results, pair k = (p, q), p <= q in the order (0,0), (0,1), (1,1), (0,2),
// (1,2), (2,2), at red[red_off + k nchunks + chunk]
template <typename P, int S>
__global__ __launch_bounds__(LS_BT) void ls_update_block_kernel(const LsArgs A)
{
    if (ls_all_ended(A)) return;
    constexpr int NG = S * (S + 1) / 2;
    __shared__ double sh[LS_BT / 64];
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& St = A.state[i];
    if (!ls_running(St)) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    const int J = St.J;
    const P* V = (const P*)A.V + I.v_off;
    P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = ls_block_vec<P>(A, q) + I.x_off;
    const double* R = A.hcol + I.hc_off;
    const int64_t r0 = ch * LS_CH, r1 = min(r0 + LS_CH, I.n);
    const int64_t n = I.vs;  // basis column stride
    double gs[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) gs[k] = 0.0;
    constexpr int E = 4;                // rows per thread: E LS_BT = LS_CH, one pass over the basis
    constexpr int CU = S <= 3 ? 4 : 2;  // basis columns per step: S CU projections held at once
    static_assert(E * LS_BT == LS_CH, "one pass per thread");
    const int64_t t0 = r0 + threadIdx.x;
    if (t0 < r1) {
        double u[S][E];
        bool in[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t t = t0 + (int64_t)e * LS_BT;
            in[e] = t < r1;
#pragma unroll
            for (int q = 0; q < S; ++q) u[q][e] = in[e] ? (double)wv[q][t] : 0.0;
        }
        int c = 0;
        for (; c + CU - 1 <= J; c += CU) {
            double h[S][CU];
#pragma unroll
            for (int q = 0; q < S; ++q)
#pragma unroll
                for (int m = 0; m < CU; ++m) h[q][m] = R[q * (J + 1) + c + m];
            const P* v0 = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e]) {
                    double a[CU];
#pragma unroll
                    for (int m = 0; m < CU; ++m) a[m] = (double)__builtin_nontemporal_load(v0 + t + m * n);  // streamed
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        double acc = h[q][0] * a[0];
#pragma unroll
                        for (int m = 1; m < CU; ++m) acc += h[q][m] * a[m];
                        u[q][e] -= acc;
                    }
                }
            }
        }
        for (; c <= J; ++c) {
            double h[S];
#pragma unroll
            for (int q = 0; q < S; ++q) h[q] = R[q * (J + 1) + c];
            const P* vc = V + (int64_t)c * n;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
                if (in[e]) {
                    const double a = (double)__builtin_nontemporal_load(vc + t);
#pragma unroll
                    for (int q = 0; q < S; ++q) u[q][e] -= h[q] * a;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (in[e]) {
                const int64_t t = t0 + (int64_t)e * LS_BT;
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
                    for (int pp = 0; pp <= q; ++pp) gs[k++] += r[pp] * r[q];
            }
        }
    }
    double* red = A.red + I.red_off;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const double v = ls_block_sum(gs[k], sh);
        if (threadIdx.x == 0) red[(int64_t)k * I.nchunks + ch] = v;
    }
}

// Rotations 0..count-1 applied to columns 0..ncol-1 (column l at base + l ld):
// lane l takes column l, the LDS loads of LS_BATCH steps issued together
__device__ void ls_rotate_cols(double* base, int ld, int ncol, int count, const double* __restrict__ cs,
                               const double* __restrict__ sn, double* sc, double* ss)
{
    const int l = threadIdx.x;
    double* colv = base + (int64_t)(l < ncol ? l : 0) * ld;
    __syncthreads();
    double a = l < ncol ? colv[0] : 0.0;
    for (int i0 = 0; i0 < count; i0 += LS_GV) {
        const int cnt = min(count - i0, LS_GV);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
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

// one block of LS_GT threads per instance: Gram sums, Cholesky (pivot i is
// resolvable when c_ii > 1e-8 sqrt(G_ii), pivot 0 when c_00 > 1e-300), the
// block's raw Hessenberg columns (Hr, leading dimension m + 2) and, rotated,
// into H; residual estimates and stop tests.  A block with p < S resolvable
// pivots takes columns J..J+p and ends the cycle; C^{-1} goes to the state for
// the normalisation.  Dynamic LDS: S columns of max_m + 4.
template <int S>
__global__ __launch_bounds__(LS_GT) void ls_block_givens_kernel(const LsArgs A, int step, int ldc)
{
    constexpr int NG = S * (S + 1) / 2;
    extern __shared__ double dyn[];
    __shared__ double sc[LS_GV], ss[LS_GV];
    __shared__ double G[S][S], Cf[S][S], Ci[S][S];  // in LDS: thread 0 indexes them dynamically
    __shared__ int ncol_s, cut_s, stop_s;
    const int i = blockIdx.x;
    LsState& St = A.state[i];
    if (!ls_running(St)) return;
    const LsInst& I = A.inst[i];
    const int j = St.J, mcyc = St.mcyc, ldh = I.m + 1, ldr = I.m + 2;
    double* H = A.H + I.H_off;
    double* Hr = A.Hr + I.Hr_off;
    double* cs = A.cs + I.h_off;
    double* sn = A.sn + I.h_off;
    double* g = A.g + I.h_off;
    const double* R = A.hcol + I.hc_off;
    const double* red = A.red + I.red_off;
    double acc[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) acc[k] = 0.0;
    if (threadIdx.x < 64) {  // the Gram partials: wave 0 (thread 0 factors them)
        for (int c = threadIdx.x; c < I.nchunks; c += 64)
#pragma unroll
            for (int k = 0; k < NG; ++k) acc[k] += red[(int64_t)k * I.nchunks + c];
#pragma unroll
        for (int k = 0; k < NG; ++k) acc[k] = ls_wave_sum(acc[k]);
    }
    for (int t = threadIdx.x; t <= j; t += LS_GT) dyn[t] = R[t] + (t == j ? A.theta : 0.0);  // Ahat v_J = w_0 + theta v_J
    if (threadIdx.x == 0) {
        int k = 0;
        for (int q = 0; q < S; ++q)
            for (int p = 0; p <= q; ++p) {
                G[p][q] = G[q][p] = acc[k];
                ++k;
            }
        int pok = 0;  // leading resolvable pivots
        for (int p = 0; p < S; ++p)
            for (int q = 0; q < S; ++q) Cf[p][q] = Ci[p][q] = 0.0;
        for (int ii = 0; ii < S; ++ii) {
            double d = G[ii][ii];
            for (int m = 0; m < ii; ++m) d -= Cf[m][ii] * Cf[m][ii];
            const double cii = d > 0.0 ? sqrt(d) : 0.0;
            const bool ok = isfinite(cii) && (ii == 0 ? cii > 1e-300 : cii > 1e-8 * sqrt(G[ii][ii]));
            Cf[ii][ii] = isfinite(cii) ? cii : 0.0;
            if (!ok) break;
            for (int q = ii + 1; q < S; ++q) {
                double v = G[ii][q];
                for (int m = 0; m < ii; ++m) v -= Cf[m][ii] * Cf[m][q];
                Cf[ii][q] = v / cii;
            }
            ++pok;
        }
        for (int ii = 0; ii < pok; ++ii) {
            Ci[ii][ii] = 1.0 / Cf[ii][ii];
            for (int q = ii + 1; q < pok; ++q) {
                double v = 0.0;
                for (int m = ii; m < q; ++m) v += Ci[ii][m] * Cf[m][q];
                Ci[ii][q] = -v / Cf[q][q];
            }
        }
        int ncol = S < mcyc - j ? S : mcyc - j;
        if (pok < S && ncol > pok + 1) ncol = pok + 1;
        ncol_s = ncol;
        cut_s = pok < S ? 1 : 0;
        dyn[j + 1] = Cf[0][0];
        for (int p = 0; p < S; ++p)
            for (int q = 0; q < S; ++q) St.ci[p * S + q] = Ci[p][q];
    }
    __syncthreads();
    const int ncol = ncol_s;
    for (int t = threadIdx.x; t <= j + 1; t += LS_GT) Hr[t + (int64_t)j * ldr] = dyn[t];
    __syncthreads();
    // columns J+1 .. J+ncol-1 from the raw column J and the earlier raw columns
    if (ncol > 1) {
        // a row per group of LS_SEG adjacent lanes: lane g of the group sums every LS_SEG-th entry of the row
        // from the g-th on (the walk along a row is a chain of dependent loads: a quarter as long), the partial
        // sums are combined by shuffles, and the group's lanes then take the columns in turn
        constexpr int SEG = LS_SEG;
        const int sg = threadIdx.x % SEG;
        for (int t = threadIdx.x / SEG; t <= j + ncol; t += LS_GT / SEG) {
            double hx[S - 1];
#pragma unroll
            for (int l = 0; l < S - 1; ++l) hx[l] = 0.0;
            if (t <= j + 1) {  // (Hr R_l)[t], loads issued HB at a time
                constexpr int HB = LS_BATCH;
                int c = (t > 0 ? t - 1 : 0) + sg;
                for (; c + SEG * (HB - 1) <= j; c += SEG * HB) {
                    double h[HB];
#pragma unroll
                    for (int u = 0; u < HB; ++u) h[u] = Hr[t + (int64_t)(c + SEG * u) * ldr];
#pragma unroll
                    for (int u = 0; u < HB; ++u)
#pragma unroll
                        for (int l = 0; l < S - 1; ++l) hx[l] += h[u] * R[l * (j + 1) + c + SEG * u];
                }
                for (; c <= j; c += SEG) {
                    const double h = Hr[t + (int64_t)c * ldr];
#pragma unroll
                    for (int l = 0; l < S - 1; ++l) hx[l] += h * R[l * (j + 1) + c];
                }
            }
#pragma unroll
            for (int l = 0; l < S - 1; ++l) {  // the group's lanes share a row and leave the loop together
#pragma unroll
                for (int o = 1; o < SEG; o *= 2) hx[l] += __shfl_xor(hx[l], o, 64);
            }
            // row t of [R; C] (coefficients on V below row j + 1, the Cholesky factor above), read once
            double rc[S];
#pragma unroll
            for (int m = 0; m < S; ++m)
                rc[m] = m >= ncol ? 0.0 : (t <= j ? R[m * (j + 1) + t] : (t - j - 1 <= m ? Cf[t - j - 1][m] : 0.0));
            double e[S - 1];  // Ahat u_l = w_{l+1} + theta w_l - Ahat V R_l, in the basis [V, Q]
#pragma unroll
            for (int l = 0; l < S - 1; ++l) e[l] = rc[l + 1] + A.theta * rc[l] - hx[l];
#pragma unroll 1
            for (int ii = 1 + sg; ii < ncol; ii += SEG) {
                if (t > j + ii + 1) continue;
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < S - 1; ++l)
                    if (l < ii) v += e[l] * Ci[l][ii - 1];
                dyn[ii * ldc + t] = v;
            }
        }
        __syncthreads();
        for (int ii = 1; ii < ncol; ++ii)
            for (int t = threadIdx.x; t <= j + ii + 1; t += LS_GT) Hr[t + (int64_t)(j + ii) * ldr] = dyn[ii * ldc + t];
    }
    // earlier blocks' rotations on all columns at once, then the columns in turn
    // (thread 0, this block's rotations and estimates in LDS: no global round
    // trip between the columns), then the columns taken written out
    ls_rotate_cols(dyn, ldc, ncol, j, cs, sn, sc, ss);
    __shared__ double bc[S], bs[S], gk[S + 1];
    __shared__ int taken_s;
    if (threadIdx.x == 0) {
        gk[0] = g[j];
        int taken = ncol, stop = 0;
        for (int ii = 0; ii < ncol; ++ii) {
            const int k = j + ii;
            double* cv = dyn + ii * ldc;
            double a = cv[j];
            for (int t = 0; t < ii; ++t) {
                const double bv = cv[j + t + 1];
                cv[j + t] = bc[t] * a + bs[t] * bv;
                a = -bs[t] * a + bc[t] * bv;
            }
            const double bv = cv[k + 1];
            const double d = sqrt(a * a + bv * bv);
            bc[ii] = d == 0.0 ? 1.0 : a / d;
            bs[ii] = d == 0.0 ? 0.0 : bv / d;
            cv[k] = d;
            gk[ii + 1] = -bs[ii] * gk[ii];
            gk[ii] = bc[ii] * gk[ii];
            if (fabs(gk[ii + 1]) <= St.cyctol || k + 1 >= mcyc || (ii == ncol - 1 && cut_s)) {
                taken = ii + 1;
                stop = 1;
                break;
            }
        }
        for (int ii = 0; ii < taken; ++ii) {
            cs[j + ii] = bc[ii];
            sn[j + ii] = bs[ii];
            g[j + ii] = gk[ii];
        }
        g[j + taken] = gk[taken];
        taken_s = taken;
        stop_s = stop;
    }
    __syncthreads();
    const int taken = taken_s;
    for (int ii = 0; ii < taken; ++ii)
        for (int t = threadIdx.x; t <= j + ii; t += LS_GT) H[t + (int64_t)(j + ii) * ldh] = dyn[ii * ldc + t];
    if (threadIdx.x == 0) {
        St.jb = j;
        St.bstep = step;
        St.J = j + taken;
        if (stop_s) {
            St.stop = 1;
            atomicSub(A.counters + 1, 1);
        }
    }
}

// q_i = sum_{l<=i} u_l (C^{-1})_{li} into V_{jb+1+i} for the instances whose
// block was taken this step, for the columns it took (t = J - jb): i <= t - 2,
// and i = t - 1 unless the cycle stopped
template <typename P, int S>
__global__ __launch_bounds__(LS_BT) void ls_normalize_block_kernel(const LsArgs A, int step)
{
    const int64_t b = blockIdx.x;
    const int i = ls_find(A.rblk, A.count, b);
    const LsState& St = A.state[i];
    if (!St.active || St.bstep != step) return;
    const int tk = St.J - St.jb;
    const int nq = St.stop ? tk - 1 : tk;
    if (nq < 1 || tk > S) return;
    const LsInst& I = A.inst[i];
    const int64_t ch = b - A.rblk[i];
    double ci[S][S];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S; ++q) ci[p][q] = St.ci[p * S + q];
    const P* wv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) wv[q] = ls_block_vec<P>(A, q) + I.x_off;
    P* out = (P*)A.V + I.v_off + (int64_t)(St.jb + 1) * I.vs;
    const int64_t r1 = min((ch + 1) * (int64_t)LS_CH, I.n);
    for (int64_t t = ch * LS_CH + threadIdx.x; t < r1; t += LS_BT) {
        double u[S];
#pragma unroll
        for (int q = 0; q < S; ++q) u[q] = (double)wv[q][t];
#pragma unroll
        for (int ii = 0; ii < S; ++ii) {
            if (ii < nq) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l <= ii; ++l) v += u[l] * ci[l][ii];
                out[(int64_t)ii * I.vs + t] = (P)v;
            }
        }
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
        for (int c = 0; c < J; ++c) s += y[c] * (double)V[(int64_t)c * I.vs + t];
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

int ls_setup(const LsArgs& A, int64_t n_eblk, int mixed, hipStream_t st)
{
    if (A.count <= 0) return DG_OK;
    const dim3 be(LS_BT), ge((unsigned)n_eblk);
    hipLaunchKernelGGL(ls_invert_kernel, ge, be, 0, st, A);
    if (mixed) hipLaunchKernelGGL((ls_form_kernel<float>), ge, be, 0, st, A);
    else hipLaunchKernelGGL((ls_form_kernel<double>), ge, be, 0, st, A);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct LsDims {
    dim3 be, ge, gr, gi;
    int max_m;
};

// the launches of one restart cycle, from the normalised residual to the
// next residual check: every Arnoldi block (numbered 1, 2, ... within the
// cycle; an instance whose cycle has ended skips the rest), the least-squares
// solve and update of x, then the true residual and the next cycle's state
template <typename P, int S>
static void ls_cycle_blocks(const LsArgs& A, const LsDims& d, hipStream_t st)
{
    const int ldc = d.max_m + 4;
    const size_t dyn = sizeof(double) * S * (size_t)ldc;
    for (int j = 0, step = 1; j < d.max_m; j += S, ++step) {
        for (int q = 0; q < S; ++q) hipLaunchKernelGGL((ls_spmv_kernel<P>), d.ge, d.be, 0, st, A, q, 1.0 - A.theta);
        if constexpr (S == 8)
            hipLaunchKernelGGL((ls_multidot_mfma_kernel<P>), d.gr, d.be, 0, st, A);
        else
            hipLaunchKernelGGL((ls_multidot_block_kernel<P, S>), d.gr, d.be, 0, st, A);
        hipLaunchKernelGGL(ls_reduce_kernel, d.gi, d.be, 0, st, A, S);
        hipLaunchKernelGGL((ls_update_block_kernel<P, S>), d.gr, d.be, 0, st, A);
        hipLaunchKernelGGL((ls_block_givens_kernel<S>), d.gi, dim3(LS_GT), dyn, st, A, step, ldc);
        hipLaunchKernelGGL((ls_normalize_block_kernel<P, S>), d.gr, d.be, 0, st, A, step);
    }
}

template <typename P>
static void ls_cycle(const LsArgs& A, const LsDims& d, hipStream_t st)
{
    hipLaunchKernelGGL((ls_cycle_init_kernel<P>), d.gr, d.be, 0, st, A);
    if (A.block == 2) ls_cycle_blocks<P, 2>(A, d, st);
    else if (A.block == 3) ls_cycle_blocks<P, 3>(A, d, st);
    else if (A.block == 6) ls_cycle_blocks<P, 6>(A, d, st);
    else if (A.block == 8) ls_cycle_blocks<P, 8>(A, d, st);
    else
        for (int j = 0; j < d.max_m; ++j) {
            hipLaunchKernelGGL((ls_spmv_kernel<P>), d.ge, d.be, 0, st, A, 0, 1.0);
            hipLaunchKernelGGL((ls_multidot_kernel<P>), d.gr, d.be, 0, st, A);
            hipLaunchKernelGGL(ls_reduce_kernel, d.gi, d.be, 0, st, A, 0);
            hipLaunchKernelGGL((ls_update_kernel<P>), d.gr, d.be, 0, st, A);
            hipLaunchKernelGGL(ls_givens_kernel, d.gi, dim3(64), 0, st, A);
            hipLaunchKernelGGL((ls_normalize_kernel<P>), d.gr, d.be, 0, st, A);
        }
    hipLaunchKernelGGL(ls_trisolve_kernel, d.gi, d.be, 0, st, A);
    hipLaunchKernelGGL((ls_combine_kernel<P>), d.gr, d.be, 0, st, A);
    hipLaunchKernelGGL((ls_dinv_update_kernel<P>), d.ge, d.be, 0, st, A);
    hipLaunchKernelGGL(ls_zero_counters, dim3(1), dim3(1), 0, st, A.counters);
    hipLaunchKernelGGL(ls_residual_kernel, d.ge, d.be, 0, st, A);
    hipLaunchKernelGGL(ls_check_kernel, d.gi, d.be, 0, st, A, 0);
}

void ls_graph_release(LsGraph& g)
{
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.cap) hipStreamDestroy(g.cap);
    g = LsGraph{};
}

// records one cycle of this chunk on the capture stream and instantiates it
template <typename P>
static int ls_record(const LsArgs& A, const LsDims& d, LsGraph& G)
{
    if (!G.cap) DG_HIP_CHECK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    if (G.exec) {
        DG_HIP_CHECK(hipGraphExecDestroy(G.exec));
        G.exec = nullptr;
    }
    G.key_x = G.key_rep = nullptr;
    DG_HIP_CHECK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    ls_cycle<P>(A, d, G.cap);
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(G.cap, &graph);
    if (le != hipSuccess || ce != hipSuccess || !graph) {
        if (graph) hipGraphDestroy(graph);
        return DG_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        G.exec = nullptr;
        return DG_ERR_HIP;
    }
    G.key_x = A.x;
    G.key_rep = A.reports;
    return DG_OK;
}

template <typename P>
static int ls_solve_p(const LsArgs& A, int64_t n_eblk, int64_t n_rblk, int max_m, hipStream_t st, dg_progress_fn fn,
                      void* user, int done_before, int total, LsGraph* graph)
{
    const LsDims d{dim3(LS_BT), dim3((unsigned)n_eblk), dim3((unsigned)n_rblk), dim3((unsigned)A.count), max_m};
    const int rs = ls_setup(A, n_eblk, A.mixed, st);
    if (rs != DG_OK) return rs;
    hipLaunchKernelGGL(ls_bnorm_kernel, d.gr, d.be, 0, st, A);
    hipLaunchKernelGGL(ls_zero_counters, dim3(1), dim3(1), 0, st, A.counters);
    hipLaunchKernelGGL(ls_residual_kernel, d.ge, d.be, 0, st, A);
    hipLaunchKernelGGL(ls_check_kernel, d.gi, d.be, 0, st, A, 1);
    DG_HIP_CHECK(hipGetLastError());
    int h[2];
    for (;;) {
        // the one host read of the cycle: instances still active after the check
        DG_HIP_CHECK(hipMemcpyAsync(h, A.counters, sizeof(h), hipMemcpyDeviceToHost, st));
        DG_HIP_CHECK(hipStreamSynchronize(st));
        if (fn) fn(user, done_before + (A.count - h[0]), total);
        if (h[0] == 0) break;
        if (graph) {
            if (!graph->exec || graph->key_x != (const void*)A.x || graph->key_rep != (const void*)A.reports) {
                const int r = ls_record<P>(A, d, *graph);
                if (r != DG_OK) return r;
            }
            DG_HIP_CHECK(hipGraphLaunch(graph->exec, st));
        } else {
            ls_cycle<P>(A, d, st);
            DG_HIP_CHECK(hipGetLastError());
        }
    }
    return DG_OK;
}

int ls_solve(const LsArgs& A, int64_t n_eblk, int64_t n_rblk, int max_m, int mixed, hipStream_t st,
             dg_progress_fn fn, void* user, int done_before, int total, LsGraph* graph)
{
    if (A.count <= 0) return DG_OK;
    return mixed ? ls_solve_p<float>(A, n_eblk, n_rblk, max_m, st, fn, user, done_before, total, graph)
                 : ls_solve_p<double>(A, n_eblk, n_rblk, max_m, st, fn, user, done_before, total, graph);
}

int64_t ls_elem_blocks(int k, int64_t T)
{
    const int n = (k + 1) * (k + 2) / 2, epw = 64 / n;
    const int64_t per = (int64_t)(LS_BT / 64) * epw;
    return (T + per - 1) / per;
}

int64_t ls_row_chunks(int64_t n) { return (n + LS_CH - 1) / LS_CH; }

}  // namespace dg
