// dg_solve_small_noalloc: block-Jacobi setup + GMRES of a small system with
// no allocation (gfx950).
//
// The same kernels as dg_solver_setup and the one-workgroup solve of
// dg_solver_solve (its Krylov state in LDS), but without a solver object: the
// setup's outputs (D^{-1} in FP64, A M^{-1} and D^{-1} in the cycle precision)
// and its failure flag live in `scratch`, a fixed device array of this file
// that every device the library runs on holds until the process ends, and the
// report goes to caller-owned device memory.  Nothing here calls hipMalloc,
// hipFree or an allocating library routine, and nothing synchronises, so a
// caller can capture the call in a HIP graph.
//
// Host code never passes `scratch` itself to a kernel: in host code that name
// is a host-side stand-in.  The first call on each device looks up the
// array's device address with hipGetSymbolAddress (with that device current)
// and keeps it; kernels get that address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "dg_internal.h"

namespace dg {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = 4u << 20;  // 4 MiB per device
constexpr size_t NOALLOC_HEAD = 256;                // setup failure flag, then the blocks
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[NOALLOC_MAX_DEVICES] = {};

// the current device's address of `scratch` (looked up once per device)
int scratch_ptr(unsigned char** out)
{
    int dev = 0;
    DG_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return DG_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        DG_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return DG_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = (unsigned char*)g_ptr[dev];
    return DG_OK;
}

// the failure flag must start at zero on every call (the array keeps the
// last call's contents); a kernel, not hipMemsetAsync, so a captured graph
// replays it correctly
__global__ void clear_flag_kernel(int* flag) { *flag = 0; }

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" int32_t dg_solve_small_noalloc(const dg_mesh* m, const dg_solver_opts* o, const double* dev_vals64,
                                          const double* dev_rhs, double* dev_x, dg_solve_report* dev_report,
                                          void* stream)
{
    if (!m || !o || !dev_vals64 || !dev_rhs || !dev_x || !dev_report) return DG_ERR_ARG;
    if (o->restart < 1 || o->restart > SMALL_MAX_RESTART || o->max_iters < 0 || !(o->rel_tol > 0) ||
        (o->mixed != 0 && o->mixed != 1) || o->reorth || o->profile)
        return DG_ERR_ARG;
    if (o->mixed && !(o->inner_tol > 0 && o->inner_tol < 1)) return DG_ERR_ARG;
    const int N = m->n;
    const int64_t T = m->T, nnzb = m->nnzb;
    const size_t ps = o->mixed ? sizeof(float) : sizeof(double);
    const size_t NN = (size_t)N * N;
    // scratch layout: flag | D^{-1} FP64 | A M^{-1} (P) | D^{-1} (P)
    const size_t off_d64 = NOALLOC_HEAD;
    const size_t off_ahat = off_d64 + align256(sizeof(double) * NN * (size_t)T);
    const size_t off_dp = off_ahat + align256(ps * NN * (size_t)std::max<int64_t>(nnzb - T, 1));
    const size_t need = off_dp + align256(ps * NN * (size_t)T);
    if (need > NOALLOC_SCRATCH_BYTES) return DG_ERR_ARG;
    const int64_t lim = small_lds_limit();
    SmallLayout L = small_layout(T, N, nnzb, o->restart, ps, true);
    if (L.bytes > lim) L = small_layout(T, N, nnzb, o->restart, ps, false);
    if (L.bytes > lim) return DG_ERR_ARG;
    unsigned char* base = nullptr;
    int r = scratch_ptr(&base);
    if (r != DG_OK) return r;
    r = small_prepare(N, o->mixed, L);
    if (r != DG_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    int* flag = (int*)base;
    double* dinv64 = (double*)(base + off_d64);
    void* ahat = base + off_ahat;
    void* dinvp = base + off_dp;
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, st, flag);
    DG_HIP_CHECK(hipGetLastError());
    r = launch_block_jacobi(N, o->mixed, dev_vals64, m->d_row_ptr, m->d_col_idx, T, dinv64, ahat, dinvp, flag, st);
    if (r != DG_OK) return r;
    SmallArgs a{};
    a.A64 = dev_vals64;
    a.rp = m->d_row_ptr;
    a.ci = m->d_col_idx;
    a.Ahat = ahat;
    a.Dinv = dinvp;
    a.b = dev_rhs;
    a.x = dev_x;
    a.rep = dev_report;
    a.bad = flag;
    a.T = T;
    a.nnzb = (int32_t)nnzb;
    a.m = o->restart;
    a.max_iters = o->max_iters;
    a.mixed = o->mixed;
    a.rel_tol = o->rel_tol;
    a.inner_tol = o->inner_tol;
    a.guess_limit = guess_limit_of(o->guess_limit);
    a.L = L;
    return small_launch(N, o->mixed, a, st);
}
