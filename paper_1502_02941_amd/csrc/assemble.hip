// Single-mesh assembly kernels (see asm_device.h for the terms computed).
#include <hip/hip_runtime.h>

#include <cmath>

#include "asm_device.h"

namespace dg {

// Thread mapping: one lane per (element K, trial function j); a wavefront
// holds floor(64 / n_loc) elements, a 256-thread block four wavefronts.
template <int K, typename R>
__global__ __launch_bounds__(256) void assemble_kernel(const AsmArgs a)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in_wave = lane / N;
    const int j = lane - e_in_wave * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e_in_wave;
    if (e_in_wave >= EPW || el >= a.T) return;
    assemble_element<K, R>(a, el, j, (R*)a.vals);
}

template <int K, typename R>
__global__ __launch_bounds__(256) void load_vector_kernel(const AsmArgs a)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in_wave = lane / N;
    const int j = lane - e_in_wave * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e_in_wave;
    if (e_in_wave >= EPW || el >= a.T) return;
    load_vector_element<K, R>(a, el, j, (R*)a.rhs);
}

template <int K, typename R>
static int launch_k(const dg_mesh* m, const AsmArgs& a, hipStream_t s)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N;
    const int64_t per_block = 4 * EPW;
    const int64_t blocks = (m->T + per_block - 1) / per_block;
    if (blocks <= 0) return DG_OK;
    if (a.vals) hipLaunchKernelGGL((assemble_kernel<K, R>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    if (a.rhs) hipLaunchKernelGGL((load_vector_kernel<K, R>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

int launch_assemble(const dg_mesh* m, const AsmArgs& a, int prec, hipStream_t s)
{
    const bool f64 = prec == DG_F64;
    switch (m->k) {
    case 0: return f64 ? launch_k<0, double>(m, a, s) : launch_k<0, float>(m, a, s);
    case 1: return f64 ? launch_k<1, double>(m, a, s) : launch_k<1, float>(m, a, s);
    case 2: return f64 ? launch_k<2, double>(m, a, s) : launch_k<2, float>(m, a, s);
    case 3: return f64 ? launch_k<3, double>(m, a, s) : launch_k<3, float>(m, a, s);
    case 4: return f64 ? launch_k<4, double>(m, a, s) : launch_k<4, float>(m, a, s);
    }
    return DG_ERR_DEGREE;
}

// Physical coordinates of the volume and boundary-edge quadrature points.
__global__ void qpoints_kernel(const double* __restrict__ xy, const double* __restrict__ tab, TabLayout L,
                               int64_t T, double* __restrict__ vol)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= T * L.nq) return;
    const int64_t K = idx / L.nq;
    const int g = (int)(idx - K * L.nq);
    const double* p = xy + 6 * K;
    const double xi = tab[L.vxi + g], eta = tab[L.veta + g];
    vol[2 * idx] = p[0] + (p[2] - p[0]) * xi + (p[4] - p[0]) * eta;
    vol[2 * idx + 1] = p[1] + (p[3] - p[1]) * xi + (p[5] - p[1]) * eta;
}

__global__ void bnd_points_kernel(const double* __restrict__ xy, const double* __restrict__ tab, TabLayout L,
                                  const int32_t* __restrict__ bel, const int32_t* __restrict__ bloc,
                                  const int32_t* __restrict__ btype, int64_t nb, double* __restrict__ pts,
                                  double* __restrict__ nrm, int32_t* __restrict__ type_out)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double* p = xy + 6 * (int64_t)bel[b];
    const int l = bloc[b];
    const double xa = p[2 * l], ya = p[2 * l + 1], xb = p[(2 * l + 2) % 6], yb = p[(2 * l + 3) % 6];
    if (pts)
        for (int g = 0; g < L.nqe; ++g) {
            const double t = tab[L.et + g];
            pts[2 * (b * L.nqe + g)] = xa + t * (xb - xa);
            pts[2 * (b * L.nqe + g) + 1] = ya + t * (yb - ya);
        }
    if (nrm) {
        const double len = sqrt((xb - xa) * (xb - xa) + (yb - ya) * (yb - ya));
        nrm[2 * b] = (yb - ya) / len;
        nrm[2 * b + 1] = -(xb - xa) / len;
    }
    if (type_out) type_out[b] = btype[b];
}

static int field_check(const dg_field& f, bool allow_points)
{
    if (f.kind < DG_CONST || f.kind > DG_QPOINTS) return DG_ERR_ARG;
    if (f.kind == DG_QPOINTS && (!allow_points || !f.dev_vals)) return DG_ERR_ARG;
    if (f.kind == DG_GAUSS_SUM && (f.m < 0 || f.m > 4)) return DG_ERR_ARG;
    const int nc = f.kind == DG_CONST ? 1 : f.kind == DG_AFFINE ? 3 : f.kind == DG_GAUSS_SUM ? 4 * f.m : 0;
    for (int i = 0; i < nc; ++i)
        if (!std::isfinite(f.c[i])) return DG_ERR_NONFINITE;
    return DG_OK;
}

static FieldDev to_affine(const dg_field& f)
{
    FieldDev d{};
    d.kind = DG_AFFINE;
    d.c[0] = f.c[0];
    d.c[1] = f.kind == DG_AFFINE ? f.c[1] : 0.0;
    d.c[2] = f.kind == DG_AFFINE ? f.c[2] : 0.0;
    return d;
}

static int affine_check(const dg_field& f)
{
    if (f.kind != DG_CONST && f.kind != DG_AFFINE) return DG_ERR_ARG;
    return field_check(f, false);
}

static FieldDev to_dev(const dg_field& f)
{
    FieldDev d;
    d.kind = f.kind;
    d.m = f.m;
    for (int i = 0; i < 16; ++i) d.c[i] = f.c[i];
    d.vals = f.dev_vals;
    return d;
}

}  // namespace dg

using namespace dg;

extern "C" int32_t dg_mesh_qpoints(const dg_mesh* m, double* dev_vol_xy, double* dev_bnd_xy, double* dev_bnd_normal,
                                   int32_t* dev_bnd_type, void* stream)
{
    if (!m) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const TabLayout L(m->k);
    if (dev_vol_xy) {
        const int64_t tot = m->T * L.nq;
        hipLaunchKernelGGL(qpoints_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m->d_xy, m->d_tab64,
                           L, m->T, dev_vol_xy);
        DG_HIP_CHECK(hipGetLastError());
    }
    if ((dev_bnd_xy || dev_bnd_normal || dev_bnd_type) && m->n_bnd > 0) {
        hipLaunchKernelGGL(bnd_points_kernel, dim3((unsigned)((m->n_bnd + 255) / 256)), dim3(256), 0, s, m->d_xy,
                           m->d_tab64, L, m->d_bnd_el, m->d_bnd_loc, m->d_bnd_type, m->n_bnd, dev_bnd_xy,
                           dev_bnd_normal, dev_bnd_type);
        DG_HIP_CHECK(hipGetLastError());
    }
    return DG_OK;
}

extern "C" int32_t dg_assemble(const dg_mesh* m, const dg_problem* P, int32_t prec, uint32_t parts, void* dev_vals,
                               void* dev_rhs, void* stream)
{
    if (!m || !P || !dev_vals) return DG_ERR_ARG;
    if (prec != DG_F64 && prec != DG_F32) return DG_ERR_ARG;
    if (parts & ~(uint32_t)DG_PART_ALL) return DG_ERR_ARG;
    if (P->degree != m->k) return DG_ERR_ARG;
    double kappa;
    switch (P->method) {
    case DG_NIPG: kappa = 1.0; break;
    case DG_SIPG: kappa = -1.0; break;
    case DG_IIPG: kappa = 0.0; break;
    default: return DG_ERR_METHOD;
    }
    if (!std::isfinite(P->sigma) || !std::isfinite(P->sigma_D) || !std::isfinite(P->b0) || P->sigma < 0)
        return DG_ERR_NONFINITE;
    int st;
    if ((st = affine_check(P->eps)) || (st = affine_check(P->bx)) || (st = affine_check(P->by)) ||
        (st = affine_check(P->alpha)) || (st = field_check(P->f, true)) || (st = field_check(P->gD, true)) ||
        (st = field_check(P->gN, true)))
        return st;
    AsmArgs a;
    a.xy = m->d_xy;
    a.nbr = m->d_nbr;
    a.nbr_edge = m->d_nbr_edge;
    a.row_ptr = m->d_row_ptr;
    a.bnd_type = m->d_bnd_type;
    a.tab = prec == DG_F64 ? (const void*)m->d_tab64 : (const void*)m->d_tab32;
    a.T = m->T;
    a.sigma = P->sigma;
    a.sigma_D = P->sigma_D > 0 ? P->sigma_D : 2.0 * P->sigma;
    a.kappa = kappa;
    a.b0 = P->b0;
    a.parts = parts;
    a.eps = to_affine(P->eps);
    a.bx = to_affine(P->bx);
    a.by = to_affine(P->by);
    a.alpha = to_affine(P->alpha);
    a.f = to_dev(P->f);
    a.gD = to_dev(P->gD);
    a.gN = to_dev(P->gN);
    a.vals = dev_vals;
    a.rhs = dev_rhs;
    return launch_assemble(m, a, prec, (hipStream_t)stream);
}
