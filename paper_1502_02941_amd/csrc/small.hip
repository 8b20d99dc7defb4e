// Restarted GMRES for a small system in one workgroup, with the whole Krylov
// state in LDS.
//
// A system of a few hundred to a few thousand unknowns leaves the chip idle
// between the ~8 launches of every Arnoldi step of the kernel-per-step solver
// (each launch costs a few microseconds, whatever its size).  Here one
// workgroup of 512 threads runs the whole solve: the basis V (restart + 1
// columns), the work vectors, the block structure, the Hessenberg matrix and
// the FP64 iterate x live in LDS (up to 160 KB on gfx950), and so do the
// operator blocks A M^{-1} formed at setup when they fit as well (else they
// and D^{-1} are read from global memory, L2 resident at these sizes); the
// host waits once per solve.
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
// and thread 0 applies the Givens rotations while the other waves run the next
// product; its stop flag is read after the next barrier (the speculative
// product is discarded).  Wave sums use DPP row operations.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "dg_internal.h"

namespace dg {

namespace {

constexpr int SBT = 512;  // threads of the solving workgroup
constexpr int SWPB = SBT / 64;

// v of the lane DPP control CTRL names (0 where that lane is outside the row
// or its row or bank is masked off), for a double split into its two words
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_double(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
    return __hiloint2double(hi, lo);
}

// sum over the 64 lanes, returned to every lane: an inclusive scan inside each
// row of 16 lanes (row shifts by 1, 2, 4, 8), the row totals carried by the
// row broadcasts of lane 15 and lane 31, and lane 63's total read out
__device__ __forceinline__ double lane_sum(double v)
{
    v += dpp_double<0x111, 0xf>(v);  // row_shr:1
    v += dpp_double<0x112, 0xf>(v);  // row_shr:2
    v += dpp_double<0x114, 0xf>(v);  // row_shr:4
    v += dpp_double<0x118, 0xf>(v);  // row_shr:8
    v += dpp_double<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_double<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
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

// A double held in lane `src` of the wavefront (src uniform), for every lane.
__device__ __forceinline__ double lane_value(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// h_c = V_c . w for the Q columns cb, cb + 8, ... of one wavefront
template <int Q, typename P>
__device__ __forceinline__ void dot_columns(const P* V, const P* w, const int n, const int lane, const int cb,
                                            double* hcol)
{
    const P* col[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) col[q] = V + (cb + q * SWPB) * n;
    double ac[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) ac[q] = 0.0;
#pragma unroll 2
    for (int t = lane; t < n; t += 64) {
        const double wv = (double)w[t];
#pragma unroll
        for (int q = 0; q < Q; ++q) ac[q] += (double)col[q][t] * wv;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) ac[q] = lane_sum(ac[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) hcol[cb + q * SWPB] = ac[q];
    }
}

// Hessenberg column j of thread 0: the earlier rotations applied to h, the new
// rotation, the residual estimate and the stop flag.  The loads of four
// rotations are issued together (the arrays do not alias), and each rotation
// puts one FMA on the dependency chain through h.
__device__ __forceinline__ void givens_column(const int j, const double hn, const bool brk, const double cyctol,
                                              const int mcyc, const double* __restrict__ hcol,
                                              double* __restrict__ hc, double* __restrict__ cs,
                                              double* __restrict__ sn, double* __restrict__ gv,
                                              int* __restrict__ flag)
{
    double av = hcol[0];
    int i = 0;
    for (; i + 4 <= j; i += 4) {
        double b[4], c[4], s[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            b[q] = hcol[i + q + 1];
            c[q] = cs[i + q];
            s[q] = sn[i + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double cb = c[q] * b[q], sb = s[q] * b[q];
            hc[i + q] = fma(c[q], av, sb);
            av = fma(-s[q], av, cb);
        }
    }
    for (; i < j; ++i) {
        const double bv = hcol[i + 1], c = cs[i], s = sn[i];
        const double cb = c * bv, sb = s * bv;
        hc[i] = fma(c, av, sb);
        av = fma(-s, av, cb);
    }
    // d = sqrt(av^2 + hn^2), c = av / d, s = hn / d, with one reciprocal square root
    const double d2 = av * av + hn * hn;
    double d, cj, sj;
    if (d2 > 0.0 && d2 <= DBL_MAX) {
        const double rd = rsqrt(d2);
        d = d2 * rd;
        cj = av * rd;
        sj = hn * rd;
    } else {
        d = sqrt(d2);
        cj = d == 0.0 ? 1.0 : av / d;
        sj = d == 0.0 ? 0.0 : hn / d;
    }
    cs[j] = cj;
    sn[j] = sj;
    hc[j] = d;
    const double g = gv[j];
    gv[j + 1] = -sj * g;
    gv[j] = cj * g;
    *flag = (fabs(sj * g) <= cyctol || brk || j + 1 >= mcyc) ? 1 : 0;
}

// STAGE: the operator blocks A M^{-1} are copied into LDS as well.
template <int N, typename P, bool STAGE>
__global__ __launch_bounds__(SBT) void small_gmres_kernel(const SmallArgs a)
{
    extern __shared__ __align__(16) char lds[];
    constexpr int EPW = 64 / N;       // elements per wavefront, lane = (element, row)
    constexpr int EPB = EPW * SWPB;   // elements per pass of the workgroup
    constexpr int EPB1 = EPW * (SWPB - 1);  // the same without wave 0
    constexpr int NN = N * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int e_in = lane / N, jj = lane - e_in * N;
    const bool lane_ok = e_in < EPW;
    // every array below lives in LDS, so 32-bit indices suffice
    const int T = (int)a.T, n = T * N;
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
    const P* Ahat = STAGE ? (const P*)(lds + L.ahat) : (const P*)a.Ahat;
    const P* Dinv = (const P*)a.Dinv;

    if (a.bad && *a.bad) {  // the setup found a singular or non-finite diagonal block
        if (tid == 0) {
            dg_solve_report rb{};
            rb.status = DG_ERR_NONFINITE;
            rb.persistent = 1;
            *a.rep = rb;
        }
        return;
    }
    for (int i = tid; i <= T; i += SBT) rp[i] = a.rp[i];
    for (int i = tid; i < a.nnzb; i += SBT) ci[i] = a.ci[i];
    if (STAGE) {
        P* dst = (P*)(lds + L.ahat);
        const P* src = (const P*)a.Ahat;
        const int cnt = (a.nnzb - T) * NN;
        for (int i = tid; i < cnt; i += SBT) dst[i] = src[i];
    }
    double acc = 0.0;
    for (int t = tid; t < n; t += SBT) {
        xs[t] = a.x[t];
        acc += a.b[t] * a.b[t];
    }
    const double bnorm = sqrt(group_sum(acc, red));  // its barriers publish rp, ci, Ahat and xs
    dg_solve_report rep{};
    rep.status = DG_NOT_CONVERGED;
    rep.persistent = 1;
    if (!isfinite(bnorm)) {
        // the caller's x is left as it was
        if (tid == 0) {
            rep.status = DG_ERR_NONFINITE;
            *a.rep = rep;
        }
        return;
    }
    if (bnorm == 0.0) {
        for (int t = tid; t < n; t += SBT) a.x[t] = 0.0;
        if (tid == 0) {
            rep.status = DG_OK;
            *a.rep = rep;
        }
        return;
    }
    // Up to degree 1, when one pass of waves 1.. covers every element, each lane
    // keeps its rows of the operator blocks and the neighbour offsets in
    // registers for the whole solve.
    constexpr bool RC = N <= 3;
    const bool regs = RC && T <= EPB1;
    P rbl[RC ? 3 : 1][RC ? N : 1];
    int rnb[3] = {-1, -1, -1};
    if constexpr (RC) {
        const int el = (wave - 1) * EPW + e_in;
        if (regs && wave > 0 && lane_ok && el < T) {
            const int s0 = rp[el], nnb = rp[el + 1] - s0 - 1, c0 = s0 - el;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                rnb[q] = q < nnb ? ci[s0 + 1 + q] * N : -1;
#pragma unroll
                for (int c = 0; c < N; ++c) rbl[q][c] = q < nnb ? Ahat[((c0 + q) * N + jj) * N + c] : (P)0;
            }
        }
    }
    const double abs_tol = a.rel_tol * bnorm;
    int its = 0;
    for (;;) {
        // ---- true FP64 residual r = F - A x ----
        acc = 0.0;
        for (int e0 = 0; e0 < T; e0 += EPB) {
            const int el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            double s = a.b[el * N + jj];
            for (int sl = rp[el]; sl < rp[el + 1]; ++sl) {
                const double* blk = a.A64 + ((int64_t)sl * N + jj) * N;
                const double* xv = xs + ci[sl] * N;
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
            for (int t = tid; t < n; t += SBT) xs[t] = 0.0;
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
        for (int t = tid; t < n; t += SBT) V[t] = (P)(r[t] * invb);
        if (tid == 0) gv[0] = beta;
        __syncthreads();

        // ---- Arnoldi steps ----
        int J = 0;
        double invh = 0.0;
        int cur = 0;
        for (int j = 0;; ++j) {
            P* vj = V + j * n;
            const P* wprev = wbuf[cur ^ 1];
            P* w = wbuf[cur];
            // w = Ahat v_j; the identity diagonal blocks are not stored.  A
            // triangle has at most three neighbours: their loads are issued
            // together.  Waves 1.. take the elements while thread 0 of wave 0
            // applies the rotations of step j - 1.
            if constexpr (RC) {
                const int el = (wave - 1) * EPW + e_in;
                if (regs && wave > 0 && lane_ok && el < T) {
                    const int row = el * N + jj;
                    double s;
                    if (j == 0) {
                        s = (double)vj[row];
                    } else {
                        const P pv = (P)((double)wprev[row] * invh);
                        vj[row] = pv;
                        s = (double)pv;
                    }
                    const P* src = j == 0 ? vj : wprev;
                    P xv[3][N];
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int c = 0; c < N; ++c) xv[q][c] = rnb[q] >= 0 ? src[rnb[q] + c] : (P)0;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (j == 0) {
#pragma unroll
                            for (int c = 0; c < N; ++c) s += (double)rbl[q][c] * (double)xv[q][c];
                        } else {
#pragma unroll
                            for (int c = 0; c < N; ++c) s += (double)rbl[q][c] * (double)(P)((double)xv[q][c] * invh);
                        }
                    }
                    w[row] = (P)s;
                }
            }
            for (int e0 = 0; e0 < T && wave > 0 && !regs; e0 += EPB1) {
                const int el = e0 + (wave - 1) * EPW + e_in;
                if (!(lane_ok && el < T)) continue;
                const int row = el * N + jj;
                double s;
                if (j == 0) {
                    s = (double)vj[row];
                } else {
                    const P pv = (P)((double)wprev[row] * invh);
                    vj[row] = pv;
                    s = (double)pv;
                }
                const int s0 = rp[el], s1 = rp[el + 1];
                const int c0 = s0 - el;
                const int nnb = s1 - s0 - 1;
                // up to degree 2 the three blocks fit the registers; above, one block at a time
                constexpr int QU = N <= 6 ? 3 : 0;
                P bl[QU > 0 ? QU : 1][N], xv[QU > 0 ? QU : 1][N];
#pragma unroll
                for (int q = 0; q < QU; ++q) {
                    if (q < nnb) {
                        const P* blk = Ahat + ((c0 + q) * N + jj) * N;
                        const P* src = (j == 0 ? vj : wprev) + ci[s0 + 1 + q] * N;
#pragma unroll
                        for (int c = 0; c < N; ++c) {
                            bl[q][c] = blk[c];
                            xv[q][c] = src[c];
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < QU; ++q) {
                    if (q < nnb) {
                        if (j == 0) {
#pragma unroll
                            for (int c = 0; c < N; ++c) s += (double)bl[q][c] * (double)xv[q][c];
                        } else {
#pragma unroll
                            for (int c = 0; c < N; ++c) s += (double)bl[q][c] * (double)(P)((double)xv[q][c] * invh);
                        }
                    }
                }
                for (int q = QU; q < nnb; ++q) {
                    const P* blk = Ahat + ((c0 + q) * N + jj) * N;
                    const int nb = ci[s0 + 1 + q] * N;
#pragma unroll
                    for (int c = 0; c < N; ++c)
                        s += (double)blk[c] * (j == 0 ? (double)vj[nb + c] : (double)(P)((double)wprev[nb + c] * invh));
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
                const int nq = min(4, (j - cb) / SWPB + 1);
                if (nq == 4) dot_columns<4>(V, w, n, lane, cb, hcol);
                else if (nq == 3) dot_columns<3>(V, w, n, lane, cb, hcol);
                else if (nq == 2) dot_columns<2>(V, w, n, lane, cb, hcol);
                else dot_columns<1>(V, w, n, lane, cb, hcol);
            }
            __syncthreads();
            // w -= V h and the partial sums of ||w||^2; h goes to registers
            // (lane l holds h_l and h_{l+64}) and is read out lane by lane
            const double hlo = lane <= j ? hcol[lane] : 0.0, hhi = lane + 64 <= j ? hcol[lane + 64] : 0.0;
            double pa = 0.0;
            for (int t = tid; t < n; t += SBT) {
                double wv = (double)w[t];
                int c = 0;
                for (; c + 3 <= j; c += 4) {
                    double h4[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) h4[q] = lane_value(c + q < 64 ? hlo : hhi, (c + q) & 63);
                    wv -= h4[0] * (double)V[c * n + t] + h4[1] * (double)V[(c + 1) * n + t] +
                          h4[2] * (double)V[(c + 2) * n + t] + h4[3] * (double)V[(c + 3) * n + t];
                }
                for (; c <= j; ++c) wv -= lane_value(c < 64 ? hlo : hhi, c & 63) * (double)V[c * n + t];
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
            double hn, rh;
            if (hn2 > 0.0 && hn2 <= DBL_MAX) {
                rh = rsqrt(hn2);
                hn = hn2 * rh;
            } else {
                hn = sqrt(hn2);  // 0, inf or NaN
                rh = 0.0;
            }
            const bool brk = !(hn > 1e-300) || !isfinite(hn);
            if (tid == 0) givens_column(j, hn, brk, cyctol, mcyc, hcol, H + j * ldh, cs, sn, gv, flag);
            invh = brk ? 0.0 : rh;
            cur ^= 1;
        }
        // y = R^{-1} g by wave 0: lane l holds g_l and g_{l+64} (restart <= 128)
        if (wave == 0) {
            double g0 = lane < J ? gv[lane] : 0.0, g1 = lane + 64 < J ? gv[lane + 64] : 0.0;
            for (int i = J - 1; i >= 0; --i) {
                const double gi = __shfl(i < 64 ? g0 : g1, i & 63, 64);
                const double yi = gi / H[i + i * ldh];
                if (lane == 0) yv[i] = yi;
                if (lane < i) g0 -= H[lane + i * ldh] * yi;
                if (lane + 64 < i) g1 -= H[lane + 64 + i * ldh] * yi;
            }
        }
        __syncthreads();
        // x += D^{-1} (V y)
        for (int t = tid; t < n; t += SBT) {
            double s = 0.0;
            for (int c = 0; c < J; ++c) s += yv[c] * (double)V[c * n + t];
            u[t] = (P)s;
        }
        __syncthreads();
        for (int e0 = 0; e0 < T; e0 += EPB) {
            const int el = e0 + wave * EPW + e_in;
            if (!(lane_ok && el < T)) continue;
            const P* d = Dinv + ((int64_t)el * N + jj) * N;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < N; ++c) s += (double)d[c] * (double)u[el * N + c];
            xs[el * N + jj] += s;
        }
        __syncthreads();
        its += J;
        rep.cycles++;
    }
    for (int t = tid; t < n; t += SBT) a.x[t] = xs[t];
    if (tid == 0) *a.rep = rep;
}

template <int N>
const void* small_kernel_fn(int mixed, bool stage)
{
    if (mixed) return stage ? (const void*)small_gmres_kernel<N, float, true> : (const void*)small_gmres_kernel<N, float, false>;
    return stage ? (const void*)small_gmres_kernel<N, double, true> : (const void*)small_gmres_kernel<N, double, false>;
}

const void* small_kernel_of(int N, int mixed, bool stage)
{
    switch (N) {
    case 1: return small_kernel_fn<1>(mixed, stage);
    case 3: return small_kernel_fn<3>(mixed, stage);
    case 6: return small_kernel_fn<6>(mixed, stage);
    case 10: return small_kernel_fn<10>(mixed, stage);
    case 15: return small_kernel_fn<15>(mixed, stage);
    }
    return nullptr;
}

}  // namespace

SmallLayout small_layout(int64_t T, int N, int64_t nnzb, int m, size_t ps, bool stage_ahat)
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
    L.ahat = stage_ahat ? take((nnzb - T) * N * N * (int64_t)ps) : -1;
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

int small_prepare(int N, int mixed, const SmallLayout& L)
{
    const void* fn = small_kernel_of(N, mixed, L.ahat >= 0);
    const int64_t lds_bytes = L.bytes;
    if (!fn) return DG_ERR_DEGREE;
    if (lds_bytes > small_lds_limit()) return DG_ERR_ARG;
    DG_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    return DG_OK;
}

int small_launch(int N, int mixed, const SmallArgs& a, hipStream_t st)
{
    const size_t sh = (size_t)a.L.bytes;
    const bool stage = a.L.ahat >= 0;
    switch (N) {
#define DG_SMALL_CASE(NN)                                                                                          \
    case NN:                                                                                                       \
        if (mixed && stage) hipLaunchKernelGGL((small_gmres_kernel<NN, float, true>), dim3(1), dim3(SBT), sh, st, a); \
        else if (mixed) hipLaunchKernelGGL((small_gmres_kernel<NN, float, false>), dim3(1), dim3(SBT), sh, st, a); \
        else if (stage) hipLaunchKernelGGL((small_gmres_kernel<NN, double, true>), dim3(1), dim3(SBT), sh, st, a); \
        else hipLaunchKernelGGL((small_gmres_kernel<NN, double, false>), dim3(1), dim3(SBT), sh, st, a);        \
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
