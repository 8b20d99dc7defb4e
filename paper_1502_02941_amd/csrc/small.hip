// Restarted GMRES for a small system in one workgroup, with the whole Krylov
// state in LDS.
//
// A system of a few hundred to a few thousand unknowns leaves the chip idle
// between the ~8 launches of every Arnoldi step of the kernel-per-step solver
// (each launch costs a few microseconds, whatever its size).  Here one
// workgroup of 512 threads runs the whole solve: the basis V (restart + 1
// columns), the work vectors, the block structure, the Hessenberg matrix and
// the FP64 iterate x live in LDS (up to 160 KB on gfx950), the operator blocks
// A M^{-1} and D^{-1} formed at setup are read from global memory (L2
// resident at these sizes), and the host waits once per solve.
//
// The algorithm is the one of the kernel-per-step solver: right block-Jacobi
// preconditioning, FP64 true residual r = F - A x per restart cycle, classical
// Gram-Schmidt Arnoldi with Givens rotations and the residual estimate, cycle
// end at the estimate target, x += D^{-1} V y in FP64, FP32 cycles with FP64
// refinement when mixed, and the residual judge of the initial guess.
//
// One Arnoldi step j takes three barriers:
//   w_j = Ahat v_j        (v_j = w_{j-1} / ||w_{j-1}||, normalised on the fly
//                          and stored as column j by the lane that owns the row)
//   h = V_{0..j}^T w_j    (each wave takes whole columns, 4 at a time)
//   w_j -= V h, ||w_j||^2 (each thread its rows; wave partials)
// and thread 0 applies the Givens rotations while the next product runs; its
// stop flag is read after the next barrier (the speculative product is
// discarded).
#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_internal.h"

namespace dg {

namespace {

constexpr int SBT = 512;  // threads of the solving workgroup
constexpr int SWPB = SBT / 64;

// sum over the 64 lanes; every lane receives the total
__device__ __forceinline__ double lane_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// workgroup sum (two barriers), returned to every thread; red holds SWPB doubles
__device__ __forceinline__ double group_sum(double v, double* red)
{
    v = lane_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < SWPB; ++w) s += red[w];
    __syncthreads();
    return s;
}

template <int N, typename P>
__global__ __launch_bounds__(SBT) void small_gmres_kernel(const SmallArgs a)
{
    extern __shared__ __align__(16) char lds[];
    constexpr int EPW = 64 / N;       // elements per wavefront, lane = (element, row)
    constexpr int EPB = EPW * SWPB;   // elements per pass of the workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e_in = lane / N, jj = lane - e_in * N;
    const bool lane_ok = e_in < EPW;
    const int64_t T = a.T, n = T * N;
    const int m = a.m, ldh = m + 1;
    const SmallLayout& L = a.L;
    P* V = (P*)(lds + L.V);
    P* wbuf[2] = {(P*)(lds + L.w0), (P*)(lds + L.w1)};
    double* r = (double*)(lds + L.r);
    P* u = (P*)(lds + L.r);  // shares r's space: r is dead once V_0 is formed
    double* xs = (double*)(lds + L.x);
    int32_t* rp = (int32_t*)(lds + L.rp);
    int32_t* ci = (int32_t*)(lds + L.ci);
    double* H = (double*)(lds + L.H);
    double* hcol = (double*)(lds + L.hcol);
    double* cs = (double*)(lds + L.cs);
    double* sn = (double*)(lds + L.sn);
    double* gv = (double*)(lds + L.gv);
    double* yv = (double*)(lds + L.yv);
    double* red = (double*)(lds + L.red);        // [SWPB] for group_sum
    double* red2 = red + SWPB;                   // [SWPB] Arnoldi norm partials
    int* flag = (int*)(lds + L.flag);
    const P* Ahat = (const P*)a.Ahat;
    const P* Dinv = (const P*)a.Dinv;

    for (int64_t i = tid; i <= T; i += SBT) rp[i] = a.rp[i];
    for (int64_t i = tid; i < a.nnzb; i += SBT) ci[i] = a.ci[i];
    double acc = 0.0;
    for (int64_t t = tid; t < n; t += SBT) {
        xs[t] = a.x[t];
        acc += a.b[t] * a.b[t];
    }
    const double bnorm = sqrt(group_sum(acc, red));  // its barriers publish rp, ci and xs
    dg_solve_report rep{};
    rep.status = DG_NOT_CONVERGED;
    if (!isfinite(bnorm)) {
        // the caller's x is left as it was
        if (tid == 0) {
            rep.status = DG_ERR_NONFINITE;
            *a.rep = rep;
        }
        return;
    }
    if (bnorm == 0.0) {
        for (int64_t t = tid; t < n; t += SBT) a.x[t] = 0.0;
        if (tid == 0) {
            rep.status = DG_OK;
            *a.rep = rep;
        }
        return;
    }
    const double abs_tol = a.rel_tol * bnorm;
    int its = 0;
    for (;;) {
        // ---- true FP64 residual r = F - A x ----
        acc = 0.0;
        for (int64_t e0 = 0; e0 < T; e0 += EPB) {
            const int64_t el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            double s = a.b[el * N + jj];
            for (int sl = rp[el]; sl < rp[el + 1]; ++sl) {
                const double* blk = a.A64 + ((int64_t)sl * N + jj) * N;
                const double* xv = xs + (int64_t)ci[sl] * N;
#pragma unroll
                for (int c = 0; c < N; ++c) s -= blk[c] * xv[c];
            }
            r[el * N + jj] = s;
            acc += s * s;
        }
        const double beta = sqrt(group_sum(acc, red));
        const double rel = beta / bnorm;
        if (rep.cycles == 0 && !rep.guess_rejected && !(rel <= a.guess_limit)) {
            // the guess is worse than zero: restart from x = 0
            for (int64_t t = tid; t < n; t += SBT) xs[t] = 0.0;
            rep.guess_rejected = 1;
            rep.rel_res0 = rel;
            __syncthreads();
            continue;
        }
        if (rep.cycles == 0 && !rep.guess_rejected) rep.rel_res0 = rel;
        rep.rel_res = rel;
        rep.iters = its;
        if (!isfinite(rel)) { rep.status = DG_ERR_NONFINITE; break; }
        if (rel <= a.rel_tol) { rep.status = DG_OK; break; }
        if (its >= a.max_iters) { rep.status = DG_NOT_CONVERGED; break; }
        const int mcyc = min(m, a.max_iters - its);
        const double cyctol = fmax(a.mixed ? a.inner_tol * beta : 0.0, abs_tol);
        const double invb = 1.0 / beta;
        for (int64_t t = tid; t < n; t += SBT) V[t] = (P)(r[t] * invb);
        if (tid == 0) gv[0] = beta;
        __syncthreads();

        // ---- Arnoldi steps ----
        int J = 0;
        double invh = 0.0;
        int cur = 0;
        for (int j = 0;; ++j) {
            P* vj = V + (int64_t)j * n;
            const P* wprev = wbuf[cur ^ 1];
            P* w = wbuf[cur];
            // w = Ahat v_j; the identity diagonal blocks are not stored
            for (int64_t e0 = 0; e0 < T; e0 += EPB) {
                const int64_t el = e0 + wave * EPW + e_in;
                if (!(lane_ok && el < T)) continue;
                const int64_t row = el * N + jj;
                double s;
                if (j == 0) {
                    s = (double)vj[row];
                } else {
                    const P pv = (P)((double)wprev[row] * invh);
                    vj[row] = pv;
                    s = (double)pv;
                }
                const int s0 = rp[el], s1 = rp[el + 1];
                const int64_t c0 = (int64_t)s0 - el;
                for (int sl = s0 + 1; sl < s1; ++sl) {
                    const P* blk = Ahat + ((c0 + (sl - s0 - 1)) * N + jj) * N;
                    const int64_t nb = (int64_t)ci[sl] * N;
                    P bl[N];
#pragma unroll
                    for (int c = 0; c < N; ++c) bl[c] = blk[c];
                    if (j == 0) {
#pragma unroll
                        for (int c = 0; c < N; ++c) s += (double)bl[c] * (double)vj[nb + c];
                    } else {
#pragma unroll
                        for (int c = 0; c < N; ++c) s += (double)bl[c] * (double)(P)((double)wprev[nb + c] * invh);
                    }
                }
                w[row] = (P)s;
            }
            __syncthreads();
            if (j > 0 && *flag) {  // Givens of step j - 1 ended the cycle: this product is discarded
                J = j;
                break;
            }
            // h_c = V_c . w, c = 0..j: wave ww takes columns ww, ww + 8, ww + 16, ww + 24, then the next 32
            for (int cb = wave; cb <= j; cb += 4 * SWPB) {
                const int cc[4] = {cb, cb + SWPB, cb + 2 * SWPB, cb + 3 * SWPB};
                const P* col[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) col[q] = V + (int64_t)min(cc[q], j) * n;
                double ac[4] = {0.0, 0.0, 0.0, 0.0};
                for (int64_t t = lane; t < n; t += 64) {
                    const double wv = (double)w[t];
#pragma unroll
                    for (int q = 0; q < 4; ++q) ac[q] += (double)col[q][t] * wv;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) ac[q] = lane_sum(ac[q]);
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (cc[q] <= j) hcol[cc[q]] = ac[q];
                }
            }
            __syncthreads();
            // w -= V h and the partial sums of ||w||^2
            double pa = 0.0;
            for (int64_t t = tid; t < n; t += SBT) {
                double wv = (double)w[t];
                int c = 0;
                for (; c + 3 <= j; c += 4)
                    wv -= hcol[c] * (double)V[(int64_t)c * n + t] + hcol[c + 1] * (double)V[(int64_t)(c + 1) * n + t] +
                          hcol[c + 2] * (double)V[(int64_t)(c + 2) * n + t] +
                          hcol[c + 3] * (double)V[(int64_t)(c + 3) * n + t];
                for (; c <= j; ++c) wv -= hcol[c] * (double)V[(int64_t)c * n + t];
                const P pv = (P)wv;
                w[t] = pv;
                pa += (double)pv * (double)pv;
            }
            pa = lane_sum(pa);
            if (lane == 0) red2[wave] = pa;
            __syncthreads();
            double hn2 = 0.0;
#pragma unroll
            for (int ww = 0; ww < SWPB; ++ww) hn2 += red2[ww];
            const double hn = sqrt(hn2);
            const bool brk = !(hn > 1e-300) || !isfinite(hn);
            if (tid == 0) {
                // Hessenberg column j: earlier rotations, the new one, the residual estimate
                double* hc = H + (int64_t)j * ldh;
                double av = hcol[0];
                for (int i = 0; i < j; ++i) {
                    const double bv = hcol[i + 1];
                    hc[i] = cs[i] * av + sn[i] * bv;
                    av = -sn[i] * av + cs[i] * bv;
                }
                const double d = sqrt(av * av + hn * hn);
                cs[j] = d == 0.0 ? 1.0 : av / d;
                sn[j] = d == 0.0 ? 0.0 : hn / d;
                hc[j] = d;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                *flag = (fabs(gv[j + 1]) <= cyctol || brk || j + 1 >= mcyc) ? 1 : 0;
            }
            invh = brk ? 0.0 : 1.0 / hn;
            cur ^= 1;
        }
        // y = R^{-1} g by wave 0: lane l holds g_l and g_{l+64} (restart <= 128)
        if (wave == 0) {
            double g0 = lane < J ? gv[lane] : 0.0, g1 = lane + 64 < J ? gv[lane + 64] : 0.0;
            for (int i = J - 1; i >= 0; --i) {
                const double gi = __shfl(i < 64 ? g0 : g1, i & 63, 64);
                const double yi = gi / H[i + (int64_t)i * ldh];
                if (lane == 0) yv[i] = yi;
                if (lane < i) g0 -= H[lane + (int64_t)i * ldh] * yi;
                if (lane + 64 < i) g1 -= H[lane + 64 + (int64_t)i * ldh] * yi;
            }
        }
        __syncthreads();
        // x += D^{-1} (V y)
        for (int64_t t = tid; t < n; t += SBT) {
            double s = 0.0;
            for (int c = 0; c < J; ++c) s += yv[c] * (double)V[(int64_t)c * n + t];
            u[t] = (P)s;
        }
        __syncthreads();
        for (int64_t e0 = 0; e0 < T; e0 += EPB) {
            const int64_t el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            const P* d = Dinv + (el * N + jj) * N;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) s += (double)d[c] * (double)u[el * N + c];
            xs[el * N + jj] += s;
        }
        __syncthreads();
        its += J;
        rep.cycles++;
    }
    for (int64_t t = tid; t < n; t += SBT) a.x[t] = xs[t];
    if (tid == 0) *a.rep = rep;
}

template <int N, typename P>
const void* small_kernel_fn()
{
    return (const void*)small_gmres_kernel<N, P>;
}

const void* small_kernel_of(int N, int mixed)
{
    switch (N) {
    case 1: return mixed ? small_kernel_fn<1, float>() : small_kernel_fn<1, double>();
    case 3: return mixed ? small_kernel_fn<3, float>() : small_kernel_fn<3, double>();
    case 6: return mixed ? small_kernel_fn<6, float>() : small_kernel_fn<6, double>();
    case 10: return mixed ? small_kernel_fn<10, float>() : small_kernel_fn<10, double>();
    case 15: return mixed ? small_kernel_fn<15, float>() : small_kernel_fn<15, double>();
    }
    return nullptr;
}

}  // namespace

SmallLayout small_layout(int64_t T, int N, int64_t nnzb, int m, size_t ps)
{
    SmallLayout L{};
    const int64_t n = T * N;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off += (bytes + 15) / 16 * 16;
        return o;
    };
    L.V = take((int64_t)(m + 1) * n * (int64_t)ps);
    L.w0 = take(n * (int64_t)ps);
    L.w1 = take(n * (int64_t)ps);
    L.r = take(n * 8);
    L.x = take(n * 8);
    L.rp = take((T + 1) * 4);
    L.ci = take(nnzb * 4);
    L.H = take((int64_t)(m + 1) * m * 8);
    L.hcol = take((int64_t)(m + 1) * 8);
    L.cs = take((int64_t)m * 8);
    L.sn = take((int64_t)m * 8);
    L.gv = take((int64_t)(m + 1) * 8);
    L.yv = take((int64_t)m * 8);
    L.red = take(2 * SWPB * 8);
    L.flag = take(16);
    L.bytes = off;
    return L;
}

int small_lds_limit()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int a = 0, b = 0;
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) a = 0;
    if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) b = 0;
    return a > b ? a : b;
}

int small_prepare(int N, int mixed, int64_t lds_bytes)
{
    const void* fn = small_kernel_of(N, mixed);
    if (!fn) return DG_ERR_DEGREE;
    if (lds_bytes > small_lds_limit()) return DG_ERR_ARG;
    DG_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    return DG_OK;
}

int small_launch(int N, int mixed, const SmallArgs& a, hipStream_t st)
{
    const size_t sh = (size_t)a.L.bytes;
    switch (N) {
#define DG_SMALL_CASE(NN)                                                                                          \
    case NN:                                                                                                       \
        if (mixed) hipLaunchKernelGGL((small_gmres_kernel<NN, float>), dim3(1), dim3(SBT), sh, st, a);          \
        else hipLaunchKernelGGL((small_gmres_kernel<NN, double>), dim3(1), dim3(SBT), sh, st, a);              \
        break;
        DG_SMALL_CASE(1)
        DG_SMALL_CASE(3)
        DG_SMALL_CASE(6)
        DG_SMALL_CASE(10)
        DG_SMALL_CASE(15)
#undef DG_SMALL_CASE
    default: return DG_ERR_DEGREE;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
