// Non-linear reaction terms and Newton's method (section 3 of Uzunca &
// Karasozen, eq. (nonlinsystem) and (newton)) on gfx950.
//
// H_i(v) = int r(u_h) phi_i and HJ_ij = int r'(u_h) phi_j phi_i are
// element-local: one lane per (element, trial function j) evaluates u_h at
// the volume points of the assembly rule and writes H_j and column j of the
// element's Jacobian block.  Newton keeps J = A + HJ in its own BSR copy whose
// off-diagonal blocks are A's (copied once) and rewrites only the diagonal
// blocks each step.  Norms are reduced in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "dg_internal.h"

namespace dg {

constexpr int NT_BLOCKS = 1024;  // fixed grid of the norm kernels

template <int K>
__global__ __launch_bounds__(256) void reaction_kernel(const double* __restrict__ xy, const double* __restrict__ tab,
                                                       int64_t T, const dg_reaction r, const double* __restrict__ x,
                                                       double* __restrict__ h, double* __restrict__ hj)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in = lane / N;
    const int j = lane - e_in * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e_in;
    if (e_in >= EPW || el >= T) return;
    const double* p = xy + 6 * el;
    const double det = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
    double xe[N];
#pragma unroll
    for (int m = 0; m < N; ++m) xe[m] = x[el * N + m];
    double hacc = 0.0;
    double jacc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) jacc[i] = 0.0;
#pragma unroll 2
    for (int g = 0; g < NQ; ++g) {
        const double* phi = tab + L.vphi + g * N;
        double u = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) u += xe[m] * phi[m];
        // r(u) = sum_p c_p u^p and r'(u) = sum_p p c_p u^(p-1)
        double rr = 0.0, dr = 0.0, up = 1.0;
        for (int q = 1; q <= r.n; ++q) {
            dr += q * r.c[q - 1] * up;
            up *= u;
            rr += r.c[q - 1] * up;
        }
        const double w = tab[L.vw + g];
        const double pj = phi[j];
        hacc += w * rr * pj;
        const double t = w * dr * pj;
#pragma unroll
        for (int i = 0; i < N; ++i) jacc[i] += t * phi[i];
    }
    if (h) h[el * N + j] = det * hacc;
    if (hj)
#pragma unroll
        for (int i = 0; i < N; ++i) hj[(el * N + i) * N + j] = det * jacc[i];
}

// y -= h (h may be NULL) and part[b] = sum of y^2 over block b's entries
__global__ __launch_bounds__(256) void sub_norm_kernel(double* __restrict__ y, const double* __restrict__ h, int64_t n,
                                                       double* __restrict__ part)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)NT_BLOCKS * 256) {
        double v = y[t];
        if (h) {
            v -= h[t];
            y[t] = v;
        }
        acc += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void sum_norm_parts_kernel(double* part)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < NT_BLOCKS; i += 256) acc += part[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[NT_BLOCKS] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// diagonal blocks of J: J[diag of el] = A[diag of el] + HJ[el]
__global__ void jacobian_diag_kernel(const double* __restrict__ A, const double* __restrict__ hj,
                                     const int32_t* __restrict__ row_ptr, int64_t T, int nn, double* __restrict__ J)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T * nn) return;
    const int64_t el = t / nn, e = t - el * nn;
    const int64_t s = (int64_t)row_ptr[el] * nn + e;
    J[s] = A[s] + hj[t];
}

__global__ void axpy_kernel(double* __restrict__ x, const double* __restrict__ w, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] += w[t];
}

static int launch_reaction(const dg_mesh* m, const dg_reaction& r, const double* x, double* h, double* hj,
                           hipStream_t s)
{
    const int N = m->n, EPW = 64 / N;
    const int64_t blocks = (m->T + 4 * EPW - 1) / (4 * EPW);
    if (blocks <= 0) return DG_OK;
    const dim3 g((unsigned)blocks), b(256);
    switch (m->k) {
    case 0: hipLaunchKernelGGL(reaction_kernel<0>, g, b, 0, s, m->d_xy, m->d_tab64, m->T, r, x, h, hj); break;
    case 1: hipLaunchKernelGGL(reaction_kernel<1>, g, b, 0, s, m->d_xy, m->d_tab64, m->T, r, x, h, hj); break;
    case 2: hipLaunchKernelGGL(reaction_kernel<2>, g, b, 0, s, m->d_xy, m->d_tab64, m->T, r, x, h, hj); break;
    case 3: hipLaunchKernelGGL(reaction_kernel<3>, g, b, 0, s, m->d_xy, m->d_tab64, m->T, r, x, h, hj); break;
    case 4: hipLaunchKernelGGL(reaction_kernel<4>, g, b, 0, s, m->d_xy, m->d_tab64, m->T, r, x, h, hj); break;
    default: return DG_ERR_DEGREE;
    }
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

static bool reaction_ok(const dg_reaction* r)
{
    if (!r || r->n < 0 || r->n > 8) return false;
    for (int i = 0; i < r->n; ++i)
        if (!std::isfinite(r->c[i])) return false;
    return true;
}

// ||y - h||^2 into host (y updated in place when h is given)
static int sub_norm(double* y, const double* h, int64_t n, double* part, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sub_norm_kernel, dim3(NT_BLOCKS), dim3(256), 0, s, y, h, n, part);
    hipLaunchKernelGGL(sum_norm_parts_kernel, dim3(1), dim3(256), 0, s, part);
    DG_HIP_CHECK(hipGetLastError());
    DG_HIP_CHECK(hipMemcpyAsync(out, part + NT_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" int32_t dg_reaction_terms(const dg_mesh* m, const dg_reaction* r, const double* dev_x, double* dev_h,
                                     double* dev_hj, void* stream)
{
    if (!m || !dev_x || !reaction_ok(r)) return DG_ERR_ARG;
    return launch_reaction(m, *r, dev_x, dev_h, dev_hj, (hipStream_t)stream);
}

extern "C" int32_t dg_newton_solve(const dg_mesh* m, const dg_reaction* r, const dg_newton_opts* o, dg_solver* solver,
                                   const double* A, const double* F, double* x, dg_newton_report* rep, void* stream)
{
    if (!m || !o || !solver || !A || !F || !x || !rep || !reaction_ok(r)) return DG_ERR_ARG;
    if (o->max_newton < 0 || !(o->tol > 0)) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int N = m->n, NN = N * N;
    const int64_t n = m->T * N;
    rep->status = DG_NOT_CONVERGED;
    rep->newton_steps = 0;
    rep->linear_iters = 0;
    rep->rel_res = NAN;
    double *J = nullptr, *hj = nullptr, *h = nullptr, *res = nullptr, *w = nullptr, *part = nullptr;
    auto al = [](double** p, size_t cnt) { return hipMalloc((void**)p, sizeof(double) * (cnt > 0 ? cnt : 1)); };
    int st = DG_OK;
    if (al(&J, (size_t)m->nnzb * NN) != hipSuccess || al(&hj, (size_t)m->T * NN) != hipSuccess ||
        al(&h, n) != hipSuccess || al(&res, n) != hipSuccess || al(&w, n) != hipSuccess ||
        al(&part, NT_BLOCKS + 1) != hipSuccess)
        st = DG_ERR_OOM;
    auto body = [&]() -> int {
        const int64_t nbz = (int64_t)m->nnzb * NN;
        DG_HIP_CHECK(hipMemcpyAsync(J, A, sizeof(double) * nbz, hipMemcpyDeviceToDevice, s));
        double f2 = 0.0;
        DG_HIP_CHECK(hipMemcpyAsync(res, F, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        int e = sub_norm(res, nullptr, n, part, &f2, s);
        if (e != DG_OK) return e;
        const double fn = std::sqrt(f2);
        if (!std::isfinite(fn)) return DG_ERR_NONFINITE;
        for (int step = 0;; ++step) {
            // -Res = F - A x - H(x)
            e = launch_reaction(m, *r, x, h, hj, s);
            if (e != DG_OK) return e;
            e = dg_residual(m, A, F, x, res, s);
            if (e != DG_OK) return e;
            double r2 = 0.0;
            e = sub_norm(res, h, n, part, &r2, s);
            if (e != DG_OK) return e;
            const double rel = fn > 0.0 ? std::sqrt(r2) / fn : std::sqrt(r2);
            rep->rel_res = rel;
            if (!std::isfinite(rel)) return DG_ERR_NONFINITE;
            if (rel <= o->tol) return DG_OK;
            if (step >= o->max_newton) return DG_NOT_CONVERGED;
            // J = A + HJ(x) on the diagonal blocks; J w = -Res from w = 0
            hipLaunchKernelGGL(jacobian_diag_kernel, dim3((unsigned)((m->T * NN + 255) / 256)), dim3(256), 0, s, A, hj,
                               m->d_row_ptr, m->T, NN, J);
            DG_HIP_CHECK(hipGetLastError());
            e = dg_solver_setup(solver, J, s);
            if (e != DG_OK) return e;
            DG_HIP_CHECK(hipMemsetAsync(w, 0, sizeof(double) * n, s));
            dg_solve_report lr{};
            e = dg_solver_solve(solver, res, w, &lr, s);
            rep->linear_iters += lr.iters;
            rep->newton_steps = step + 1;
            if (e < 0) return e;
            hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, w, n);
            DG_HIP_CHECK(hipGetLastError());
        }
    };
    if (st == DG_OK) st = body();
    hipStreamSynchronize(s);
    solver_invalidate(solver);  // it was set up on J, freed below
    hipFree(J); hipFree(hj); hipFree(h); hipFree(res); hipFree(w); hipFree(part);
    rep->status = st;
    return st;
}
