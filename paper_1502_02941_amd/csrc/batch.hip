// Batched DG assembly + block-Jacobi GMRES in one persistent launch (gfx950).
//
// Many independent instances (own mesh, degree 1 or 2, coefficients and
// data) are assembled and solved by two stream-ordered launches:
//   1. batch_assemble_kernel: FP64 assembly of the matrix and load vector of
//      section 1 eq. (ds), section 2.3 eq. (system) for every element of every
//      instance in one element-parallel grid (the same per-element device
//      functions as the single-mesh kernels), into per-instance segments;
//   2. batch_kernel, persistent: one workgroup per workspace slot; each
//      workgroup takes the next instance from a queue ordered by decreasing
//      estimated cost (an atomic counter: every workgroup leaves the loop once
//      the queue is empty, so the grid drains) and runs, with workgroup
//      barriers between phases:
//   2a. block-Jacobi setup: FP64 inverse of every diagonal block, A D^{-1}
//      without its identity blocks and D^{-1} in the cycle precision P;
//   3. restarted GMRES on A D^{-1} with classical Gram-Schmidt, FP64 true
//      residual r = F - A x before every cycle, cycles in P (FP32 cycles +
//      FP64 residual / update = iterative refinement), until
//      ||F - A x|| / ||F|| <= tol or the iteration cap.
// The solution is written to the instance's segment of x (which holds the
// initial guess on entry) and a report to reports[instance].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

#include "asm_device.h"
#include "lockstep.h"

namespace dg {

constexpr int B_MAXM = 512;  // largest restart length per instance
constexpr int B_CT = 16;     // Gram-Schmidt dot products reduced together

struct BatchInst {
    int64_t el_off, rp_off, ci_off, bnd_off, x_off, val_off, blk_off;
    int64_t T, nnzb;
    int32_t k, m;
};

struct SlotPtrs {
    double* r;
    double* Dinv64;
    void* Ahat;
    void* Dinv;
    void* V;
    void* w;
    void* u;
    double* H;  // (B_MAXM+1) x B_MAXM column-major
};

struct BatchArgs {
    const BatchInst* inst;
    const AsmArgs* args;  // per instance: assembly arguments with device pointers
    const int32_t* order;
    int32_t count;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const SlotPtrs* slots;
    double* x;
    const double* A64;  // concatenated FP64 matrices
    const double* rhs;  // concatenated load vectors
    int* queue;
    dg_solve_report* reports;
    double rel_tol, inner_tol, guess_limit;
    int32_t max_iters, mixed;
};

template <int BT>
struct BatchSmem {
    double red[BT / 64][B_CT];
    double hcol[B_MAXM + 2];
    double cs[B_MAXM], sn[B_MAXM], gv[B_MAXM + 1], yv[B_MAXM];
    double bc[4];
    int flag[4];
    int q;
};

__device__ __forceinline__ double bwave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// sum over the workgroup, returned to every thread
template <int BT>
__device__ __forceinline__ double wg_sum(double v, BatchSmem<BT>& sm)
{
    v = bwave_sum(v);
    if ((threadIdx.x & 63) == 0) sm.red[threadIdx.x >> 6][0] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < BT / 64; ++w) t += sm.red[w][0];
        sm.bc[0] = t;
    }
    __syncthreads();
    const double r = sm.bc[0];
    __syncthreads();
    return r;
}

// Gauss-Jordan inverse with partial pivoting of an N x N block held by N
// lanes (lane gb + r holds row r in m[]).  Pivot rows are found and broadcast
// with wavefront shuffles; a row interchange only swaps the lanes' row labels.
// On return the lane labelled lr holds row lr of the inverse.  Returns false
// (uniformly for the group) if a pivot is zero or not finite.
template <int N>
__device__ __forceinline__ bool invert_rows(double (&m)[N], const int r, const int gb, int& lr)
{
    lr = r;
    int pc[N];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        // pivot: largest |m[c]| among rows labelled >= c (ties: lowest label)
        double best = -1.0;
        int bl = -1, blabel = N;
#pragma unroll
        for (int t = 0; t < N; ++t) {
            const double v = fabs(__shfl(m[c], gb + t, 64));
            const int lt = __shfl(lr, gb + t, 64);
            if (lt >= c && (v > best || (v == best && lt < blabel))) { best = v; bl = t; blabel = lt; }
        }
        pc[c] = blabel;
        if (!(best > 0.0) || !isfinite(best)) ok = false;
        // the lane labelled c and the pivot lane swap labels
        const int holder = [&]() {
            int h = 0;
#pragma unroll
            for (int t = 0; t < N; ++t) if (__shfl(lr, gb + t, 64) == c) h = t;
            return h;
        }();
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
    // undo the interchanges as column interchanges, last pivot first
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

// 2a. Block-Jacobi setup of one instance by the whole workgroup, lane =
// (element, row): the FP64 inverse of every diagonal block into Dinv64, then
// A D^{-1} without its identity diagonal blocks into Ahat ([nnzb - T][N][N],
// block row order) and D^{-1} into DinvP (skipped when null), both in the
// cycle precision P.  Returns false, uniformly over the workgroup, when a
// pivot of some block was zero or not finite (Ahat is then not formed).
template <int K, typename P, int BT>
__device__ bool batch_setup(const double* __restrict__ A64, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ ci, const int64_t T, double* __restrict__ Dinv64,
                            P* __restrict__ Ahat, P* __restrict__ DinvP, BatchSmem<BT>& sm)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N, WPB = BT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e_in = lane / N, jj = lane - e_in * N;
    const bool lane_ok = e_in < EPW;
    if (tid == 0) sm.flag[1] = 0;
    __syncthreads();
    for (int64_t e0 = 0; e0 < T; e0 += (int64_t)WPB * EPW) {
        const int64_t el = e0 + wave * EPW + e_in;
        const bool act = lane_ok && el < T;
        double mrow[N];
        const double* D = A64 + ((int64_t)(act ? rp[el] : 0) * N + jj) * N;
#pragma unroll
        for (int q = 0; q < N; ++q) mrow[q] = act ? D[q] : (q == jj ? 1.0 : 0.0);
        int lr;
        // every lane of the wavefront takes part in the shuffles; idle lanes invert the identity
        const bool ok = invert_rows<N>(mrow, jj, lane_ok ? e_in * N : (lane / N) * N, lr);
        if (act) {
            if (!ok) sm.flag[1] = 1;
            double* o = Dinv64 + (el * N + lr) * N;
#pragma unroll
            for (int q = 0; q < N; ++q) o[q] = mrow[q];
        }
    }
    __syncthreads();
    if (sm.flag[1]) return false;  // the flag is next written after the caller's next barrier
    for (int64_t e0 = 0; e0 < T; e0 += (int64_t)WPB * EPW) {
        const int64_t el = e0 + wave * EPW + e_in;
        if (!(lane_ok && el < T)) continue;
        const int i = jj;
        const int s0 = rp[el], s1 = rp[el + 1];
        const int64_t c0 = (int64_t)s0 - el;
        for (int sl = s0 + 1; sl < s1; ++sl) {
            const double* arow = A64 + ((int64_t)sl * N + i) * N;
            const double* d = Dinv64 + (int64_t)ci[sl] * N * N;
            P* out = Ahat + ((c0 + (sl - s0 - 1)) * N + i) * N;
            double ar[N];
#pragma unroll
            for (int k2 = 0; k2 < N; ++k2) ar[k2] = arow[k2];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                double s = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) s += ar[k2] * d[k2 * N + c];
                out[c] = (P)s;
            }
        }
        if (DinvP) {
            const double* dd = Dinv64 + (el * N + i) * N;
#pragma unroll
            for (int c = 0; c < N; ++c) DinvP[(el * N + i) * N + c] = (P)dd[c];
        }
    }
    __syncthreads();
    return true;
}

template <int K, typename P, int BT>
__device__ void run_instance(const BatchArgs& A, const BatchInst& I, const int id, const SlotPtrs& S,
                             BatchSmem<BT>& sm)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N, WPB = BT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e_in = lane / N, jj = lane - e_in * N;
    const bool lane_ok = e_in < EPW;
    const int64_t T = I.T, n = T * N;
    const int32_t* rp = A.row_ptr + I.rp_off;
    const int32_t* ci = A.col_idx + I.ci_off;
    double* x = A.x + I.x_off;
    P* V = (P*)S.V;
    P* w = (P*)S.w;
    P* u = (P*)S.u;
    const P* Ahat = (const P*)S.Ahat;
    P* DinvP = (P*)S.Dinv;
    const int ldh = B_MAXM + 1;

    const double* A64 = A.A64 + I.val_off;
    const double* rhs = A.rhs + I.x_off;
    // ---- 2. block-Jacobi setup ----
    if (!batch_setup<K, P, BT>(A64, rp, ci, T, S.Dinv64, (P*)S.Ahat, DinvP, sm)) {
        if (tid == 0) {
            dg_solve_report r{};
            r.status = DG_ERR_NONFINITE;
            A.reports[id] = r;
        }
        __syncthreads();
        return;
    }

    // ---- 3. GMRES cycles ----
    double acc = 0.0;
    for (int64_t t = tid; t < n; t += BT) acc += rhs[t] * rhs[t];
    const double bnorm = sqrt(wg_sum<BT>(acc, sm));
    dg_solve_report rep{};
    rep.status = DG_NOT_CONVERGED;
    if (!(bnorm > 0.0) || !isfinite(bnorm)) {
        for (int64_t t = tid; t < n; t += BT) x[t] = 0.0;
        rep.status = isfinite(bnorm) ? DG_OK : DG_ERR_NONFINITE;
        if (tid == 0) A.reports[id] = rep;
        __syncthreads();
        return;
    }
    const double abs_tol = A.rel_tol * bnorm;
    int its = 0;
    for (;;) {
        // true FP64 residual
        acc = 0.0;
        for (int64_t e0 = 0; e0 < T; e0 += (int64_t)WPB * EPW) {
            const int64_t el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            double s = rhs[el * N + jj];
            for (int sl = rp[el]; sl < rp[el + 1]; ++sl) {
                const double* blk = A64 + ((int64_t)sl * N + jj) * N;
                const double* xv = x + (int64_t)ci[sl] * N;
#pragma unroll
                for (int c = 0; c < N; ++c) s -= blk[c] * xv[c];
            }
            S.r[el * N + jj] = s;
            acc += s * s;
        }
        const double beta = sqrt(wg_sum<BT>(acc, sm));
        const double rel = beta / bnorm;
        if (rep.cycles == 0 && !rep.guess_rejected && !(rel <= A.guess_limit)) {
            // the guess is worse than zero: restart from x = 0
            for (int64_t t = tid; t < n; t += BT) x[t] = 0.0;
            rep.guess_rejected = 1;
            rep.rel_res0 = rel;
            __syncthreads();
            continue;
        }
        if (rep.cycles == 0 && !rep.guess_rejected) rep.rel_res0 = rel;
        rep.rel_res = rel;
        rep.iters = its;
        if (!isfinite(rel)) { rep.status = DG_ERR_NONFINITE; break; }
        if (rel <= A.rel_tol) { rep.status = DG_OK; break; }
        if (its >= A.max_iters) { rep.status = DG_NOT_CONVERGED; break; }
        const int mcyc = min(I.m, A.max_iters - its);
        const double cyctol = fmax(A.mixed ? A.inner_tol * beta : 0.0, abs_tol);
        const double invb = 1.0 / beta;
        for (int64_t t = tid; t < n; t += BT) V[t] = (P)(S.r[t] * invb);
        if (tid == 0) sm.gv[0] = beta;
        __syncthreads();
        int J = 0;
        for (int j = 0; j < mcyc; ++j) {
            const P* vj = V + (int64_t)j * n;
            // w = Ahat v_j (identity diagonal blocks)
            for (int64_t e0 = 0; e0 < T; e0 += (int64_t)WPB * EPW) {
                const int64_t el = e0 + wave * EPW + e_in;
                if (!(lane_ok && el < T)) continue;
                const int s0 = rp[el], s1 = rp[el + 1];
                const int64_t c0 = (int64_t)s0 - el;
                double s = (double)vj[el * N + jj];
                for (int sl = s0 + 1; sl < s1; ++sl) {
                    const P* blk = Ahat + ((c0 + (sl - s0 - 1)) * N + jj) * N;
                    const P* xv = vj + (int64_t)ci[sl] * N;
#pragma unroll
                    for (int c = 0; c < N; ++c) s += (double)blk[c] * (double)xv[c];
                }
                w[el * N + jj] = (P)s;
            }
            __syncthreads();
            // h = V^T w and ||w||^2 (column j+1), B_CT columns per reduction
            const int ncols = j + 2;
            for (int t0 = 0; t0 < ncols; t0 += B_CT) {
                const P* col[B_CT];
#pragma unroll
                for (int c = 0; c < B_CT; ++c) col[c] = (t0 + c <= j) ? V + (int64_t)(t0 + c) * n : w;
                double ac[B_CT];
#pragma unroll
                for (int c = 0; c < B_CT; ++c) ac[c] = 0.0;
                for (int64_t t = tid; t < n; t += BT) {
                    const double wv = (double)w[t];
#pragma unroll
                    for (int c = 0; c < B_CT; ++c) ac[c] += (double)col[c][t] * wv;
                }
#pragma unroll
                for (int c = 0; c < B_CT; ++c) {
                    const double v = bwave_sum(ac[c]);
                    if (lane == 0) sm.red[wave][c] = v;
                }
                __syncthreads();
                if (tid < B_CT && t0 + tid < ncols) {
                    double s = 0.0;
                    for (int ww = 0; ww < WPB; ++ww) s += sm.red[ww][tid];
                    sm.hcol[t0 + tid] = s;
                }
                __syncthreads();
            }
            // w -= V h, ||w||^2
            acc = 0.0;
            for (int64_t t = tid; t < n; t += BT) {
                double wv = (double)w[t];
                int c = 0;
                for (; c + 3 <= j; c += 4)
                    wv -= sm.hcol[c] * (double)V[(int64_t)c * n + t] + sm.hcol[c + 1] * (double)V[(int64_t)(c + 1) * n + t] +
                          sm.hcol[c + 2] * (double)V[(int64_t)(c + 2) * n + t] +
                          sm.hcol[c + 3] * (double)V[(int64_t)(c + 3) * n + t];
                for (; c <= j; ++c) wv -= sm.hcol[c] * (double)V[(int64_t)c * n + t];
                const P pv = (P)wv;
                w[t] = pv;
                acc += (double)pv * (double)pv;
            }
            const double hn = sqrt(wg_sum<BT>(acc, sm));
            // Hessenberg column, Givens rotations, estimate, stop test
            if (tid == 0) {
                double* hc = S.H + (int64_t)j * ldh;
                double av = sm.hcol[0];
                for (int i = 0; i < j; ++i) {
                    const double bv = sm.hcol[i + 1];
                    hc[i] = sm.cs[i] * av + sm.sn[i] * bv;
                    av = -sm.sn[i] * av + sm.cs[i] * bv;
                }
                const double d = sqrt(av * av + hn * hn);
                sm.cs[j] = d == 0.0 ? 1.0 : av / d;
                sm.sn[j] = d == 0.0 ? 0.0 : hn / d;
                hc[j] = d;
                sm.gv[j + 1] = -sm.sn[j] * sm.gv[j];
                sm.gv[j] = sm.cs[j] * sm.gv[j];
                const bool brk = !(hn > 1e-300) || !isfinite(hn);
                sm.flag[0] = (fabs(sm.gv[j + 1]) <= cyctol || brk || j + 1 >= mcyc) ? 1 : 0;
                sm.bc[1] = brk ? 0.0 : 1.0 / hn;
            }
            __syncthreads();
            J = j + 1;
            if (sm.flag[0]) break;
            const P sc = (P)sm.bc[1];
            P* vn = V + (int64_t)(j + 1) * n;
            for (int64_t t = tid; t < n; t += BT) vn[t] = w[t] * sc;
            __syncthreads();
        }
        // y = R^{-1} g
        for (int i = J - 1; i >= 0; --i) {
            if (tid == 0) sm.yv[i] = sm.gv[i] / S.H[i + (int64_t)i * ldh];
            __syncthreads();
            const double yi = sm.yv[i];
            for (int k2 = tid; k2 < i; k2 += BT) sm.gv[k2] -= S.H[k2 + (int64_t)i * ldh] * yi;
            __syncthreads();
        }
        // x += D^{-1} (V y)
        for (int64_t t = tid; t < n; t += BT) {
            double s = 0.0;
            for (int c = 0; c < J; ++c) s += sm.yv[c] * (double)V[(int64_t)c * n + t];
            u[t] = (P)s;
        }
        __syncthreads();
        for (int64_t e0 = 0; e0 < T; e0 += (int64_t)WPB * EPW) {
            const int64_t el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            const P* d = DinvP + (el * N + jj) * N;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) s += (double)d[c] * (double)u[el * N + c];
            x[el * N + jj] += s;
        }
        __syncthreads();
        its += J;
        rep.cycles++;
    }
    if (tid == 0) A.reports[id] = rep;
    __syncthreads();
}

// Element-parallel assembly of every instance: block b belongs to the
// instance i with blk_off[i] <= b < blk_off[i+1] (binary search); lanes map to
// (element, trial function) as in the single-mesh kernel.
__global__ __launch_bounds__(256) void batch_assemble_kernel(const BatchInst* __restrict__ inst,
                                                             const AsmArgs* __restrict__ args, int32_t count,
                                                             double* __restrict__ A64, double* __restrict__ rhs)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (inst[mid].blk_off <= b) lo = mid;
        else hi = mid - 1;
    }
    const BatchInst& I = inst[lo];
    const AsmArgs& a = args[lo];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (I.k == 1) {
        constexpr int N = 3, EPW = 64 / N;
        const int e_in = lane / N, j = lane - e_in * N;
        const int64_t el = ((b - I.blk_off) * 4 + wave) * EPW + e_in;
        if (e_in >= EPW || el >= I.T) return;
        assemble_element<1, double>(a, el, j, A64 + I.val_off);
        load_vector_element<1, double>(a, el, j, rhs + I.x_off);
    } else {
        constexpr int N = 6, EPW = 64 / N;
        const int e_in = lane / N, j = lane - e_in * N;
        const int64_t el = ((b - I.blk_off) * 4 + wave) * EPW + e_in;
        if (e_in >= EPW || el >= I.T) return;
        assemble_element<2, double>(a, el, j, A64 + I.val_off);
        load_vector_element<2, double>(a, el, j, rhs + I.x_off);
    }
}

template <typename P, int BT>
__global__ __launch_bounds__(BT) void batch_kernel(const BatchArgs A)
{
    __shared__ BatchSmem<BT> sm;
    const SlotPtrs S = A.slots[blockIdx.x];
    for (;;) {
        // system scope: the host reads the counter as progress while the grid runs
        if (threadIdx.x == 0) sm.q = __hip_atomic_fetch_add(A.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __syncthreads();
        const int q = sm.q;
        __syncthreads();
        if (q >= A.count) break;
        const int id = A.order[q];
        const BatchInst& I = A.inst[id];
        if (I.k == 1) run_instance<1, P, BT>(A, I, id, S, sm);
        else run_instance<2, P, BT>(A, I, id, S, sm);
    }
}

// The block-Jacobi setup of one persistent-path instance again, by the same
// device function and on the same FP64 values, into caller buffers (the
// slots keep only the last instance each ran).
template <typename P, int BT>
__global__ __launch_bounds__(BT) void batch_setup_kernel(const BatchArgs A, int id, double* Dinv64, P* Ahat)
{
    __shared__ BatchSmem<BT> sm;
    const BatchInst& I = A.inst[id];
    const double* A64 = A.A64 + I.val_off;
    const int32_t* rp = A.row_ptr + I.rp_off;
    const int32_t* ci = A.col_idx + I.ci_off;
    if (I.k == 1) batch_setup<1, P, BT>(A64, rp, ci, I.T, Dinv64, Ahat, (P*)nullptr, sm);
    else batch_setup<2, P, BT>(A64, rp, ci, I.T, Dinv64, Ahat, (P*)nullptr, sm);
}

__global__ void reset_queue_kernel(int* q) { __hip_atomic_store(q, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM); }

}  // namespace dg

using namespace dg;

struct dg_batch {
    int32_t count = 0;
    dg_batch_opts o{};
    int nslots = 0;
    std::vector<int64_t> x_off;  // [count + 1]
    // device
    BatchInst* d_inst = nullptr;
    AsmArgs* d_args = nullptr;
    int32_t* d_order = nullptr;
    double* d_xy = nullptr;
    int32_t *d_nbr = nullptr, *d_nbr_edge = nullptr, *d_rp = nullptr, *d_ci = nullptr, *d_bt = nullptr;
    double *d_tab1 = nullptr, *d_tab2 = nullptr;
    SlotPtrs* d_slots = nullptr;
    std::vector<void*> slot_mem;
    int* d_queue = nullptr;
    hipStream_t progress_stream = nullptr;
    double* d_A64 = nullptr;
    double* d_rhs = nullptr;
    int64_t total_blocks = 0, total_vals = 0;
    // persistent part: instances below the size threshold, in queue order
    int32_t n_persistent = 0;
    // lockstep part: chunks of large instances
    struct Chunk {
        int32_t count = 0;
        int64_t n_eblk = 0, n_rblk = 0;
        int max_m = 0;
        LsInst* d_inst = nullptr;
        LsState* d_state = nullptr;
        int64_t* d_eblk = nullptr;
        int64_t* d_rblk = nullptr;
        LsGraph graph;  // its restart cycle as a HIP graph (unless opts.lockstep_eager)
    };
    std::vector<Chunk> chunks;
    void *ls_V = nullptr, *ls_Ahat = nullptr, *ls_DinvP = nullptr, *ls_w = nullptr, *ls_w1 = nullptr, *ls_w2 = nullptr;
    void* ls_wx[LS_SMAX - 3] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double* ls_Hr = nullptr;
    double *ls_Dinv64 = nullptr, *ls_part = nullptr, *ls_red = nullptr, *ls_red2 = nullptr, *ls_hcol = nullptr;
    double *ls_H = nullptr, *ls_cs = nullptr, *ls_sn = nullptr, *ls_g = nullptr, *ls_y = nullptr, *ls_r = nullptr;
    int* ls_counters = nullptr;
    dg_progress_fn progress_fn = nullptr;
    void* progress_user = nullptr;
    // per instance: lockstep chunk (-1: persistent path) and offsets of its
    // inverse diagonal blocks and A D^{-1} in the chunk buffers
    std::vector<int32_t> where_chunk;
    std::vector<int64_t> where_dinv, where_ahat;
    std::vector<BatchInst> h_inst;  // host copy of d_inst
    int64_t ran = 0;  // dg_batch_run calls so far
};

// Arnoldi vectors per Gram-Schmidt pass of the lockstep solver (automatic:
// eight; on the 64 x 64 P1 family eight beat three and six in both precisions)
static int lockstep_block_of(const dg_batch_opts& o) { return o.lockstep_block != 0 ? o.lockstep_block : 8; }

static void batch_free(dg_batch* b)
{
    hipFree(b->d_inst); hipFree(b->d_args); hipFree(b->d_order); hipFree(b->d_xy); hipFree(b->d_nbr); hipFree(b->d_nbr_edge);
    hipFree(b->d_rp); hipFree(b->d_ci); hipFree(b->d_bt); hipFree(b->d_tab1); hipFree(b->d_tab2);
    hipFree(b->d_slots); hipFree(b->d_queue); hipFree(b->d_A64); hipFree(b->d_rhs);
    if (b->progress_stream) hipStreamDestroy(b->progress_stream);
    for (void* p : b->slot_mem) hipFree(p);
    b->slot_mem.clear();
    for (auto& c : b->chunks) {
        ls_graph_release(c.graph);
        hipFree(c.d_inst); hipFree(c.d_state); hipFree(c.d_eblk); hipFree(c.d_rblk);
    }
    b->chunks.clear();
    hipFree(b->ls_V); hipFree(b->ls_Ahat); hipFree(b->ls_DinvP); hipFree(b->ls_w); hipFree(b->ls_Dinv64);
    hipFree(b->ls_part); hipFree(b->ls_red); hipFree(b->ls_red2); hipFree(b->ls_hcol); hipFree(b->ls_H);
    hipFree(b->ls_cs); hipFree(b->ls_sn); hipFree(b->ls_g); hipFree(b->ls_y); hipFree(b->ls_r);
    hipFree(b->ls_w1); hipFree(b->ls_w2); hipFree(b->ls_Hr);
    for (void* p : b->ls_wx) hipFree(p);
    hipFree(b->ls_counters);
}

template <typename T>
static int up(T** dst, const T* src, size_t count)
{
    if (hipMalloc((void**)dst, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) { *dst = nullptr; return DG_ERR_OOM; }
    if (count && hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return DG_ERR_HIP;
    return DG_OK;
}

static FieldDev fdev(const dg_field& f, bool affine_only)
{
    FieldDev d{};
    d.kind = affine_only ? DG_AFFINE : f.kind;
    d.m = f.m;
    for (int i = 0; i < 16; ++i) d.c[i] = f.c[i];
    if (affine_only && f.kind == DG_CONST) d.c[1] = d.c[2] = 0.0;
    d.vals = nullptr;
    return d;
}

static int check_field(const dg_field& f, bool allow_gauss)
{
    if (f.kind == DG_CONST || f.kind == DG_AFFINE) {
        const int nc = f.kind == DG_CONST ? 1 : 3;
        for (int i = 0; i < nc; ++i)
            if (!std::isfinite(f.c[i])) return DG_ERR_NONFINITE;
        return DG_OK;
    }
    if (f.kind == DG_GAUSS_SUM && allow_gauss) {
        if (f.m < 0 || f.m > 4) return DG_ERR_ARG;
        for (int i = 0; i < 4 * f.m; ++i)
            if (!std::isfinite(f.c[i])) return DG_ERR_NONFINITE;
        return DG_OK;
    }
    return DG_ERR_ARG;
}

extern "C" int32_t dg_batch_create(const dg_instance* in, int32_t count, const dg_batch_opts* o, dg_batch** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (!in || count <= 0 || !o) return DG_ERR_ARG;
    if (o->block_threads != 0 && o->block_threads != 256 && o->block_threads != 512) return DG_ERR_ARG;
    if (o->lockstep_block < 0 || o->lockstep_block > 8 || o->lockstep_block == 4 || o->lockstep_block == 5 ||
        o->lockstep_block == 7)
        return DG_ERR_ARG;
    if (o->lockstep_basis < 0 || o->lockstep_basis > 2) return DG_ERR_ARG;
    if (o->lockstep_eager != 0 && o->lockstep_eager != 1) return DG_ERR_ARG;
    if (o->restart_max < 1 || o->restart_max > B_MAXM || o->restart_min < 1 || !(o->rel_tol > 0) ||
        o->max_iters < 0 || (o->mixed != 0 && o->mixed != 1) || (o->mixed && !(o->inner_tol > 0 && o->inner_tol < 1)))
        return DG_ERR_ARG;
    // host preprocessing, instances in parallel
    std::vector<dg_mesh> meshes(count);
    std::vector<int> st(count, DG_OK);
    {
        const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (int i = t; i < count; i += nth) {
                    const dg_instance& I = in[i];
                    const dg_problem& P = I.problem;
                    if (P.degree < 1 || P.degree > 2) { st[i] = DG_ERR_DEGREE; continue; }
                    if (P.method != DG_NIPG && P.method != DG_SIPG && P.method != DG_IIPG) { st[i] = DG_ERR_METHOD; continue; }
                    int s = DG_OK;
                    if ((s = check_field(P.eps, false)) || (s = check_field(P.bx, false)) ||
                        (s = check_field(P.by, false)) || (s = check_field(P.alpha, false)) ||
                        (s = check_field(P.f, true)) || (s = check_field(P.gD, false)) || (s = check_field(P.gN, false))) {
                        st[i] = s;
                        continue;
                    }
                    st[i] = build_host_mesh(I.nodes_xy, I.n_nodes, I.elems, I.n_elems, I.dir_edges, I.n_dir,
                                            I.neu_edges, I.n_neu, P.degree, &meshes[i], false);
                }
            });
        for (auto& t : th) t.join();
    }
    for (int i = 0; i < count; ++i)
        if (st[i] != DG_OK) return st[i];
    dg_batch* b = new (std::nothrow) dg_batch();
    if (!b) return DG_ERR_OOM;
    b->count = count;
    b->o = *o;
    // concatenate
    std::vector<BatchInst> hinst(count);
    int64_t tot_el = 0, tot_rp = 0, tot_ci = 0, tot_bnd = 0, tot_x = 0, tot_val = 0, tot_blk = 0;
    b->x_off.resize(count + 1);
    size_t need_vec = 0, need_dinv = 0, need_ahat = 0, need_V = 0;
    std::vector<size_t> i_vec(count), i_dinv(count), i_ahat(count), i_V(count);
    const size_t ps = o->mixed ? sizeof(float) : sizeof(double);
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
        const dg_mesh& m = meshes[i];
        const dg_problem& P = in[i].problem;
        BatchInst& I = hinst[i];
        I.el_off = tot_el; I.rp_off = tot_rp; I.ci_off = tot_ci; I.bnd_off = tot_bnd; I.x_off = tot_x;
        I.val_off = tot_val; I.blk_off = tot_blk;
        tot_val += m.nnzb * (int64_t)m.n * m.n;
        tot_blk += (m.T + 4 * (64 / m.n) - 1) / (4 * (64 / m.n));
        I.T = m.T; I.nnzb = m.nnzb; I.k = m.k;
        const double side = std::sqrt((double)m.T / 2.0);
        I.m = (int)std::min<double>(o->restart_max, std::max<double>(1.0, o->restart_min + o->restart_per_side * side));
        b->x_off[i] = tot_x;
        tot_el += m.T; tot_rp += m.T + 1; tot_ci += m.nnzb; tot_bnd += std::max<int64_t>(m.n_bnd, 1);
        const int64_t dofs = m.T * m.n;
        tot_x += dofs;
        const size_t NN = (size_t)m.n * m.n;
        i_vec[i] = (size_t)dofs;
        i_dinv[i] = (size_t)m.T * NN;
        i_ahat[i] = (size_t)(m.nnzb - m.T) * NN;
        i_V[i] = (size_t)(I.m + 1) * dofs;
        cost[i] = (double)I.m * I.m * dofs + 50.0 * m.nnzb * NN;
    }
    b->x_off[count] = tot_x;
    b->total_blocks = tot_blk;
    b->total_vals = tot_val;
    std::vector<int32_t> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return cost[p] > cost[q]; });
    // instances with at least lockstep_min_dofs unknowns go to the lockstep solver
    std::vector<int32_t> pers, lock;
    for (int32_t id : order)
        (b->x_off[id + 1] - b->x_off[id] >= o->lockstep_min_dofs ? lock : pers).push_back(id);
    b->n_persistent = (int32_t)pers.size();
    order = pers;  // the persistent queue
    order.insert(order.end(), lock.begin(), lock.end());
    std::vector<double> xy(6 * tot_el);
    std::vector<int32_t> nbr(3 * tot_el), nbe(tot_el), rp(tot_rp), ci(tot_ci), bt(tot_bnd, 0);
    for (int i = 0; i < count; ++i) {
        const dg_mesh& m = meshes[i];
        const BatchInst& I = hinst[i];
        std::copy(m.xy6.begin(), m.xy6.end(), xy.begin() + 6 * I.el_off);
        std::copy(m.nbr.begin(), m.nbr.end(), nbr.begin() + 3 * I.el_off);
        std::copy(m.nbr_edge.begin(), m.nbr_edge.end(), nbe.begin() + I.el_off);
        std::copy(m.row_ptr.begin(), m.row_ptr.end(), rp.begin() + I.rp_off);
        std::copy(m.col_idx.begin(), m.col_idx.end(), ci.begin() + I.ci_off);
        std::copy(m.bnd_type.begin(), m.bnd_type.end(), bt.begin() + I.bnd_off);
    }
    meshes.clear();
    std::vector<double> t1 = build_tables(1, DG_BASIS_DUBINER), t2 = build_tables(2, DG_BASIS_DUBINER);
    int s = DG_OK;
    if (s == DG_OK) s = up(&b->d_inst, hinst.data(), hinst.size());
    b->h_inst = hinst;
    if (s == DG_OK) s = up(&b->d_order, order.data(), order.size());
    if (s == DG_OK) s = up(&b->d_xy, xy.data(), xy.size());
    if (s == DG_OK) s = up(&b->d_nbr, nbr.data(), nbr.size());
    if (s == DG_OK) s = up(&b->d_nbr_edge, nbe.data(), nbe.size());
    if (s == DG_OK) s = up(&b->d_rp, rp.data(), rp.size());
    if (s == DG_OK) s = up(&b->d_ci, ci.data(), ci.size());
    if (s == DG_OK) s = up(&b->d_bt, bt.data(), bt.size());
    if (s == DG_OK) s = up(&b->d_tab1, t1.data(), t1.size());
    if (s == DG_OK) s = up(&b->d_tab2, t2.data(), t2.size());
    if (s == DG_OK && hipMalloc((void**)&b->d_queue, sizeof(int)) != hipSuccess) s = DG_ERR_OOM;
    if (s == DG_OK && hipMalloc((void**)&b->d_A64, sizeof(double) * std::max<int64_t>(tot_val, 1)) != hipSuccess)
        s = DG_ERR_OOM;
    if (s == DG_OK && hipMalloc((void**)&b->d_rhs, sizeof(double) * std::max<int64_t>(tot_x, 1)) != hipSuccess)
        s = DG_ERR_OOM;
    if (s == DG_OK) {
        std::vector<AsmArgs> args(count);
        for (int i = 0; i < count; ++i) {
            const dg_problem& P = in[i].problem;
            const BatchInst& I = hinst[i];
            AsmArgs& a = args[i];
            a.xy = b->d_xy + 6 * I.el_off;
            a.nbr = b->d_nbr + 3 * I.el_off;
            a.nbr_edge = b->d_nbr_edge + I.el_off;
            a.row_ptr = b->d_rp + I.rp_off;
            a.bnd_type = b->d_bt + I.bnd_off;
            a.tab = I.k == 1 ? (const void*)b->d_tab1 : (const void*)b->d_tab2;
            a.T = I.T;
            a.sigma = P.sigma;
            a.sigma_D = P.sigma_D > 0 ? P.sigma_D : 2.0 * P.sigma;
            a.kappa = P.method == DG_NIPG ? 1.0 : (P.method == DG_SIPG ? -1.0 : 0.0);
            a.b0 = P.b0;
            a.parts = DG_PART_ALL;
            a.eps = fdev(P.eps, true); a.bx = fdev(P.bx, true); a.by = fdev(P.by, true);
            a.alpha = fdev(P.alpha, true);
            a.f = fdev(P.f, false); a.gD = fdev(P.gD, false); a.gN = fdev(P.gN, false);
            a.vals = nullptr;
            a.rhs = nullptr;
        }
        s = up(&b->d_args, args.data(), args.size());
    }
    // workspace slots
    int ncu = 0;
    if (s == DG_OK) {
        hipDeviceProp_t prop;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) s = DG_ERR_HIP;
        else ncu = prop.multiProcessorCount;
    }
    for (int32_t id : pers) {
        need_vec = std::max(need_vec, i_vec[id]);
        need_dinv = std::max(need_dinv, i_dinv[id]);
        need_ahat = std::max(need_ahat, i_ahat[id]);
        need_V = std::max(need_V, i_V[id]);
    }
    b->nslots = o->slots > 0 ? o->slots : std::max(1, ncu);
    b->nslots = std::min(b->nslots, std::max(b->n_persistent, 0));
    std::vector<SlotPtrs> slots(std::max(b->nslots, 0));
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t szv8 = align(need_vec * 8), szD64 = align(need_dinv * 8),
                 szAh = align(std::max<size_t>(need_ahat, 1) * ps), szDp = align(need_dinv * ps),
                 szV = align(need_V * ps), szvp = align(need_vec * ps),
                 szH = align((size_t)(B_MAXM + 1) * B_MAXM * 8);
    const size_t slot_bytes = szv8 + szD64 + szAh + szDp + szV + 2 * szvp + szH;
    for (int sl = 0; sl < b->nslots && s == DG_OK; ++sl) {
        char* p = nullptr;
        if (hipMalloc((void**)&p, slot_bytes) != hipSuccess) { s = DG_ERR_OOM; break; }
        b->slot_mem.push_back(p);
        SlotPtrs& S = slots[sl];
        S.r = (double*)p; p += szv8;
        S.Dinv64 = (double*)p; p += szD64;
        S.Ahat = p; p += szAh;
        S.Dinv = p; p += szDp;
        S.V = p; p += szV;
        S.w = p; p += szvp;
        S.u = p; p += szvp;
        S.H = (double*)p;
    }
    if (s == DG_OK && b->nslots > 0) s = up(&b->d_slots, slots.data(), slots.size());
    // lockstep chunks: cost order, greedy under the memory budget
    b->where_chunk.assign(count, -1);
    b->where_dinv.assign(count, 0);
    b->where_ahat.assign(count, 0);
    if (s == DG_OK && !lock.empty()) {
        const double budget = (o->lockstep_mem_gb > 0 ? o->lockstep_mem_gb : 64.0) * 1e9;
        // partials, projections and Gram sums sized for blocks of lsb vectors
        // (at least two: the one-vector path fits in the same room)
        const int lsb = lockstep_block_of(*o) < 2 ? 2 : lockstep_block_of(*o);
        const size_t lsg = (size_t)lsb * (lsb + 1) / 2;
        size_t mx_dinv = 0, mx_ahat = 0, mx_V = 0, mx_part = 0, mx_red = 0, mx_red2 = 0, mx_hc = 0, mx_h = 0, mx_H = 0;
        size_t mx_Hr = 0;
        size_t i0 = 0;
        while (i0 < lock.size() && s == DG_OK) {
            size_t i1 = i0, dinv = 0, ahat = 0, V = 0, part = 0, red = 0, red2 = 0, hc = 0, hh = 0, H = 0, Hr = 0;
            double bytes = 0.0;
            std::vector<LsInst> li;
            std::vector<int64_t> eb(1, 0), rb(1, 0);
            int max_m = 0;
            while (i1 < lock.size()) {
                const int id = lock[i1];
                const BatchInst& I = hinst[id];
                const int N = (I.k + 1) * (I.k + 2) / 2;
                const int64_t n = I.T * N;
                const int64_t nch = ls_row_chunks(n), neb = ls_elem_blocks(I.k, I.T);
                const size_t nV = (size_t)(I.m + 1) * ls_vstride(n);  // the basis with aligned columns
                const double add = (double)nV * ps + (double)i_ahat[id] * ps + (double)i_dinv[id] * (8 + ps) +
                                   (double)(I.m + 2) * nch * 8 * lsb + (double)lsg * nch * 8 +
                                   (double)(I.m + 1) * (I.m + 6) * 8 +
                                   (double)(I.m + 2) * (I.m + 1) * 8;
                if (!li.empty() && bytes + add > budget) break;
                LsInst L{};
                L.T = I.T; L.n = n; L.vs = ls_vstride(n); L.k = I.k; L.m = I.m; L.id = id; L.id_local = (int32_t)li.size();
                L.nchunks = (int32_t)nch; L.neblk = (int32_t)neb;
                L.rp_off = I.rp_off; L.ci_off = I.ci_off; L.val_off = I.val_off; L.x_off = I.x_off;
                L.dinv_off = dinv; L.ahat_off = ahat; L.v_off = V; L.part_off = part;
                L.red_off = red; L.red2_off = red2; L.hc_off = hc; L.h_off = hh; L.H_off = H; L.Hr_off = Hr;
                // lsb (m + 2) columns of partials, lsb (lsb + 1) / 2 Gram sums per row chunk
                dinv += i_dinv[id]; ahat += i_ahat[id]; V += nV; part += (size_t)lsb * (I.m + 2) * nch;
                red += lsg * (size_t)nch; red2 += neb; hc += (size_t)lsb * ((size_t)I.m + 2); hh += I.m + 1;
                H += (size_t)(I.m + 1) * I.m; Hr += (size_t)(I.m + 2) * (I.m + 1);
                eb.push_back(eb.back() + neb);
                rb.push_back(rb.back() + nch);
                max_m = std::max(max_m, (int)I.m);
                bytes += add;
                li.push_back(L);
                b->where_chunk[id] = (int32_t)b->chunks.size();
                b->where_dinv[id] = L.dinv_off;
                b->where_ahat[id] = L.ahat_off;
                ++i1;
            }
            dg_batch::Chunk c;
            c.count = (int32_t)li.size();
            c.n_eblk = eb.back();
            c.n_rblk = rb.back();
            c.max_m = max_m;
            if (s == DG_OK) s = up(&c.d_inst, li.data(), li.size());
            if (s == DG_OK) s = up(&c.d_eblk, eb.data(), eb.size());
            if (s == DG_OK) s = up(&c.d_rblk, rb.data(), rb.size());
            if (s == DG_OK && hipMalloc((void**)&c.d_state, sizeof(LsState) * c.count) != hipSuccess) s = DG_ERR_OOM;
            b->chunks.push_back(c);
            mx_dinv = std::max(mx_dinv, dinv); mx_ahat = std::max(mx_ahat, ahat); mx_V = std::max(mx_V, V);
            mx_part = std::max(mx_part, part); mx_red = std::max(mx_red, red); mx_red2 = std::max(mx_red2, red2);
            mx_hc = std::max(mx_hc, hc); mx_h = std::max(mx_h, hh); mx_H = std::max(mx_H, H);
            mx_Hr = std::max(mx_Hr, Hr);
            i0 = i1;
        }
        auto al = [&](void** p, size_t bytes) {
            if (s == DG_OK && hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) { *p = nullptr; s = DG_ERR_OOM; }
        };
        al(&b->ls_V, mx_V * ps);
        al(&b->ls_Ahat, mx_ahat * ps);
        al(&b->ls_DinvP, mx_dinv * ps);
        al((void**)&b->ls_Dinv64, mx_dinv * 8);
        al(&b->ls_w, (size_t)tot_x * ps);
        al(&b->ls_w1, (size_t)tot_x * ps);
        if (lsb >= 3) al(&b->ls_w2, (size_t)tot_x * ps);
        for (int q = 3; q < lsb; ++q) al(&b->ls_wx[q - 3], (size_t)tot_x * ps);
        al((void**)&b->ls_Hr, mx_Hr * 8);
        al((void**)&b->ls_r, (size_t)tot_x * 8);
        al((void**)&b->ls_part, mx_part * 8);
        al((void**)&b->ls_red, mx_red * 8);
        al((void**)&b->ls_red2, mx_red2 * 8);
        al((void**)&b->ls_hcol, mx_hc * 8);
        al((void**)&b->ls_H, mx_H * 8);
        al((void**)&b->ls_cs, mx_h * 8);
        al((void**)&b->ls_sn, mx_h * 8);
        al((void**)&b->ls_g, mx_h * 8);
        al((void**)&b->ls_y, mx_h * 8);
        al((void**)&b->ls_counters, 2 * sizeof(int));
    }
    if (s != DG_OK) { batch_free(b); delete b; return s; }
    *out = b;
    return DG_OK;
}

extern "C" int32_t dg_batch_offsets(const dg_batch* b, int64_t* x_offsets)
{
    if (!b || !x_offsets) return DG_ERR_ARG;
    std::copy(b->x_off.begin(), b->x_off.end(), x_offsets);
    return DG_OK;
}

static BatchArgs batch_args(const dg_batch* b, double* dev_x, dg_solve_report* dev_reports)
{
    BatchArgs A;
    A.inst = b->d_inst;
    A.args = b->d_args;
    A.order = b->d_order;
    A.count = b->n_persistent;
    A.row_ptr = b->d_rp;
    A.col_idx = b->d_ci;
    A.slots = b->d_slots;
    A.x = dev_x;
    A.A64 = b->d_A64;
    A.rhs = b->d_rhs;
    A.queue = b->d_queue;
    A.reports = dev_reports;
    A.rel_tol = b->o.rel_tol;
    A.guess_limit = guess_limit_of(b->o.guess_limit);
    A.inner_tol = b->o.inner_tol;
    A.max_iters = b->o.max_iters;
    A.mixed = b->o.mixed;
    return A;
}

static LsArgs ls_args(const dg_batch* b, const dg_batch::Chunk& c, double* dev_x, dg_solve_report* dev_reports)
{
    LsArgs L{};
    L.count = c.count;
    L.inst = c.d_inst;
    L.state = c.d_state;
    L.eblk = c.d_eblk;
    L.rblk = c.d_rblk;
    L.row_ptr = b->d_rp;
    L.col_idx = b->d_ci;
    L.A64 = b->d_A64;
    L.rhs = b->d_rhs;
    L.x = dev_x;
    L.r = b->ls_r;
    L.w = b->ls_w;
    L.w1 = b->ls_w1;
    L.w2 = b->ls_w2;
    for (int q = 0; q < LS_SMAX - 3; ++q) L.wx[q] = b->ls_wx[q];
    L.theta = b->o.lockstep_basis == 1 ? 0.0 : 1.0;
    L.Hr = b->ls_Hr;
    L.block = lockstep_block_of(b->o);
    L.V = b->ls_V;
    L.Ahat = b->ls_Ahat;
    L.DinvP = b->ls_DinvP;
    L.Dinv64 = b->ls_Dinv64;
    L.part = b->ls_part;
    L.red = b->ls_red;
    L.red2 = b->ls_red2;
    L.hcol = b->ls_hcol;
    L.H = b->ls_H;
    L.cs = b->ls_cs;
    L.sn = b->ls_sn;
    L.g = b->ls_g;
    L.y = b->ls_y;
    L.reports = dev_reports;
    L.counters = b->ls_counters;
    L.rel_tol = b->o.rel_tol;
    L.guess_limit = guess_limit_of(b->o.guess_limit);
    L.inner_tol = b->o.inner_tol;
    L.max_iters = b->o.max_iters;
    L.mixed = b->o.mixed;
    return L;
}

extern "C" int32_t dg_batch_run(dg_batch* b, double* dev_x, dg_solve_report* dev_reports, void* stream)
{
    if (!b || !dev_x || !dev_reports) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const BatchArgs A = batch_args(b, dev_x, dev_reports);
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, st, b->d_queue);
    hipLaunchKernelGGL(batch_assemble_kernel, dim3((unsigned)b->total_blocks), dim3(256), 0, st,
                       (const BatchInst*)b->d_inst, (const AsmArgs*)b->d_args, b->count, b->d_A64, b->d_rhs);
    b->ran++;
    const int bt = b->o.block_threads ? b->o.block_threads : 512;
    if (b->n_persistent > 0) {
        if (b->o.mixed) {
            if (bt == 256) hipLaunchKernelGGL((batch_kernel<float, 256>), dim3(b->nslots), dim3(256), 0, st, A);
            else hipLaunchKernelGGL((batch_kernel<float, 512>), dim3(b->nslots), dim3(512), 0, st, A);
        } else {
            if (bt == 256) hipLaunchKernelGGL((batch_kernel<double, 256>), dim3(b->nslots), dim3(256), 0, st, A);
            else hipLaunchKernelGGL((batch_kernel<double, 512>), dim3(b->nslots), dim3(512), 0, st, A);
        }
        DG_HIP_CHECK(hipGetLastError());
    }
    int done = 0;
    for (auto& c : b->chunks) {
        const LsArgs L = ls_args(b, c, dev_x, dev_reports);
        int r = ls_init(L, st);
        if (r == DG_OK) r = ls_solve(L, c.n_eblk, c.n_rblk, c.max_m, b->o.mixed, st, b->progress_fn, b->progress_user,
                                     done, b->count - b->n_persistent, b->o.lockstep_eager ? nullptr : &c.graph);
        if (r != DG_OK) return r;
        done += c.count;
    }
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_batch_system(const dg_batch* b, int32_t instance, double* dev_vals64, double* dev_rhs,
                                   void* stream)
{
    if (!b || instance < 0 || instance >= b->count || b->ran == 0) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const BatchInst& I = b->h_inst[instance];
    const int64_t N = (I.k + 1) * (I.k + 2) / 2;
    if (dev_vals64)
        DG_HIP_CHECK(hipMemcpyAsync(dev_vals64, b->d_A64 + I.val_off, sizeof(double) * I.nnzb * N * N,
                                    hipMemcpyDeviceToDevice, st));
    if (dev_rhs)
        DG_HIP_CHECK(hipMemcpyAsync(dev_rhs, b->d_rhs + I.x_off, sizeof(double) * I.T * N, hipMemcpyDeviceToDevice, st));
    return DG_OK;
}

extern "C" int32_t dg_batch_preconditioner(dg_batch* b, int32_t instance, double* dev_dinv64, void* dev_ahat,
                                           void* stream)
{
    if (!b || instance < 0 || instance >= b->count || b->ran == 0 || !dev_dinv64 || !dev_ahat) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const BatchInst& I = b->h_inst[instance];
    const int64_t N = (I.k + 1) * (I.k + 2) / 2;
    const size_t ps = b->o.mixed ? sizeof(float) : sizeof(double);
    const int ci = b->where_chunk[instance];
    if (ci < 0) {
        const BatchArgs A = batch_args(b, nullptr, nullptr);
        const int bt = b->o.block_threads ? b->o.block_threads : 512;
        if (b->o.mixed) {
            if (bt == 256)
                hipLaunchKernelGGL((batch_setup_kernel<float, 256>), dim3(1), dim3(256), 0, st, A, instance, dev_dinv64,
                                   (float*)dev_ahat);
            else
                hipLaunchKernelGGL((batch_setup_kernel<float, 512>), dim3(1), dim3(512), 0, st, A, instance, dev_dinv64,
                                   (float*)dev_ahat);
        } else {
            if (bt == 256)
                hipLaunchKernelGGL((batch_setup_kernel<double, 256>), dim3(1), dim3(256), 0, st, A, instance,
                                   dev_dinv64, (double*)dev_ahat);
            else
                hipLaunchKernelGGL((batch_setup_kernel<double, 512>), dim3(1), dim3(512), 0, st, A, instance,
                                   dev_dinv64, (double*)dev_ahat);
        }
        DG_HIP_CHECK(hipGetLastError());
        return DG_OK;
    }
    const dg_batch::Chunk& c = b->chunks[ci];
    const LsArgs L = ls_args(b, c, nullptr, nullptr);
    const int r = ls_setup(L, c.n_eblk, b->o.mixed, st);
    if (r != DG_OK) return r;
    DG_HIP_CHECK(hipMemcpyAsync(dev_dinv64, b->ls_Dinv64 + b->where_dinv[instance], sizeof(double) * I.T * N * N,
                                hipMemcpyDeviceToDevice, st));
    if (I.nnzb > I.T)
        DG_HIP_CHECK(hipMemcpyAsync(dev_ahat, (char*)b->ls_Ahat + ps * b->where_ahat[instance],
                                    ps * (I.nnzb - I.T) * N * N, hipMemcpyDeviceToDevice, st));
    return DG_OK;
}

extern "C" int32_t dg_batch_set_progress(dg_batch* b, dg_progress_fn fn, void* user)
{
    if (!b) return DG_ERR_ARG;
    b->progress_fn = fn;
    b->progress_user = user;
    return DG_OK;
}

extern "C" int32_t dg_batch_progress(dg_batch* b, int32_t* started)
{
    if (!b || !started) return DG_ERR_ARG;
    if (!b->progress_stream && hipStreamCreateWithFlags(&b->progress_stream, hipStreamNonBlocking) != hipSuccess)
        return DG_ERR_HIP;
    int v = 0;
    DG_HIP_CHECK(hipMemcpyAsync(&v, b->d_queue, sizeof(int), hipMemcpyDeviceToHost, b->progress_stream));
    DG_HIP_CHECK(hipStreamSynchronize(b->progress_stream));
    *started = std::min(v, b->n_persistent);
    return DG_OK;
}

extern "C" void dg_batch_destroy(dg_batch* b)
{
    if (!b) return;
    batch_free(b);
    delete b;
}
