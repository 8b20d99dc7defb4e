// Backward Euler in time on the GPU.  Section 3 obtains its stationary
// problem from a time discretisation: the linear reaction coefficient alpha
// stands for 1/dt.  One step from u^n solves the system of the mesh with
// alpha = alpha_0 + 1/dt and the load vector F + (1/dt) M u^n, M the mass
// matrix, for u^{n+1} (by Newton's method when the problem has the non-linear
// reaction r(u)), starting from u^n.
//
// With the orthonormal reference basis (the integral of phi_i phi_j over the
// reference triangle is delta_ij) the mass matrix of element K is
// |det J_K| times the identity, so M u^n is an element-wise scaling; with the
// monomials it is |det J_K| times the reference Gram matrix G.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_internal.h"

namespace dg {
namespace {

constexpr int EB = 256;

// out = F + inv_dt * M u: dof t of element K = t / N
__global__ __launch_bounds__(EB) void euler_rhs_kernel(const double* __restrict__ xy, const double* __restrict__ F,
                                                       const double* __restrict__ u, double inv_dt, int N, int64_t n,
                                                       double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (t >= n) return;
    const double* p = xy + 6 * (t / N);
    const double det = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
    out[t] = F[t] + inv_dt * det * u[t];
}

// the same with a full reference mass matrix G [N][N]: (M u)_t = det sum_j G[i][j] u_(K, j)
__global__ __launch_bounds__(EB) void euler_rhs_gram_kernel(const double* __restrict__ xy, const double* __restrict__ F,
                                                            const double* __restrict__ u, double inv_dt, int N,
                                                            int64_t n, const double* __restrict__ G,
                                                            double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (t >= n) return;
    const int64_t K = t / N;
    const int i = (int)(t - K * N);
    const double* p = xy + 6 * K;
    const double det = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += G[i * N + j] * u[K * N + j];
    out[t] = F[t] + inv_dt * det * s;
}

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" int32_t dg_euler_rhs(const dg_mesh* m, const double* F, const double* u, double inv_dt, double* out,
                                void* stream)
{
    if (!m || !F || !u || !out || !std::isfinite(inv_dt)) return DG_ERR_ARG;
    const int64_t n = m->T * m->n;
    if (n == 0) return DG_OK;
    if (m->basis == DG_BASIS_MONOMIAL)
        hipLaunchKernelGGL(euler_rhs_gram_kernel, dim3((unsigned)((n + EB - 1) / EB)), dim3(EB), 0,
                           (hipStream_t)stream, m->d_xy, F, u, inv_dt, m->n, n, (const double*)m->d_mref, out);
    else
        hipLaunchKernelGGL(euler_rhs_kernel, dim3((unsigned)((n + EB - 1) / EB)), dim3(EB), 0, (hipStream_t)stream,
                           m->d_xy, F, u, inv_dt, m->n, n, out);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_implicit_euler(const dg_mesh* m, const dg_reaction* r, const dg_newton_opts* nopts,
                                     dg_solver* solver, const double* A, const double* F, double inv_dt,
                                     int32_t n_steps, double* x, dg_euler_report* rep, void* stream)
{
    if (!m || !solver || !A || !F || !x || !rep || n_steps < 0 || !(inv_dt > 0) || !std::isfinite(inv_dt))
        return DG_ERR_ARG;
    if (r && !nopts) return DG_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    *rep = dg_euler_report{};
    rep->status = DG_OK;
    const int64_t n = m->T * m->n;
    double* rhs = nullptr;
    if (hipMalloc((void**)&rhs, sizeof(double) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) return DG_ERR_OOM;
    int status = DG_OK;
    if (!r) status = dg_solver_setup(solver, A, stream);
    for (int32_t step = 0; step < n_steps && status == DG_OK; ++step) {
        status = dg_euler_rhs(m, F, x, inv_dt, rhs, stream);
        if (status != DG_OK) break;
        if (r) {
            dg_newton_report nr{};
            status = dg_newton_solve(m, r, nopts, solver, A, rhs, x, &nr, stream);
            rep->newton_steps += nr.newton_steps;
            rep->linear_iters += nr.linear_iters;
            rep->rel_res = nr.rel_res;
        } else {
            dg_solve_report sr{};
            status = dg_solver_solve(solver, rhs, x, &sr, stream);
            rep->linear_iters += sr.iters;
            rep->rel_res = sr.rel_res;
        }
        if (status == DG_OK) rep->steps = step + 1;
    }
    if (hipStreamSynchronize(st) != hipSuccess && status == DG_OK) status = DG_ERR_HIP;
    hipFree(rhs);
    rep->status = status;
    return status;
}
