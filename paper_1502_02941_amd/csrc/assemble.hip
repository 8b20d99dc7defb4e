// Element-centric assembly of the interior penalty DG system on gfx950.
//
// Computes, for every element K, block row K of D + C + R (section 2.3 eq.
// (dgscheme), (system) of Uzunca & Karasozen) and the load vector entries
// F_i = l_h(phi_i) of section 1 eq. (ds):
//   volume:   eps grad phi_j . grad phi_i + (b . grad phi_j) phi_i + alpha phi_j phi_i,  f phi_i
//   interior edge e = K cap L (n = outward normal of K, beta = b . n):
//     (K,K): -1/2 eps (grad phi_j.n) phi_i + kappa/2 eps (grad phi_i.n) phi_j
//            + (sigma eps / |e|^b0 + max(-beta,0)) phi_j phi_i
//     (K,L): -1/2 eps (grad psi_j.n) phi_i - kappa/2 eps (grad phi_i.n) psi_j
//            - (sigma eps / |e|^b0 + max(-beta,0)) psi_j phi_i        (psi = basis of L)
//   Dirichlet edge: -eps (grad phi_j.n) phi_i + kappa eps (grad phi_i.n) phi_j
//            + (sigma_D eps / |e|^b0 + max(-beta,0)) phi_j phi_i;
//     load:  g^D ((sigma_D eps / |e|^b0 + max(-beta,0)) phi_i + kappa eps grad phi_i.n)
//   Neumann edge: load g^N phi_i only.
// The interior-edge terms are the jump / average form of eq. (ds) with
// [v] = (v_K - v_L) n and {w} = (w_K + w_L)/2 written from K's side; the
// upwind term is the element-wise form over the inflow part of dK, decided per
// quadrature point.  Every block of block row K is written by the threads of
// element K only (atomic-free; each interior edge is integrated from both
// sides), so the output is bitwise deterministic.
//
// Thread mapping: one lane per (element K, trial function j); a wavefront
// holds floor(64 / n_loc) elements.  Each lane accumulates column j of the
// diagonal block and of the three neighbour blocks in registers.  The loops
// run over quadrature points g and test functions i with wave-uniform
// indices, so the test-function table values are scalar loads, while the
// per-lane work is the trial function's data at g.  Column j of each block is
// written by lane j: the n_loc lanes of an element write contiguous rows.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dg_internal.h"

namespace dg {

template <typename R>
__device__ __forceinline__ R field_at(const FieldDev& F, R x, R y, int64_t pidx)
{
    switch (F.kind) {
    case DG_CONST: return (R)F.c[0];
    case DG_AFFINE: return (R)F.c[0] + (R)F.c[1] * x + (R)F.c[2] * y;
    case DG_GAUSS_SUM: {
        R s = 0;
        for (int i = 0; i < F.m; ++i) {
            const R dx = x - (R)F.c[4 * i], dy = y - (R)F.c[4 * i + 1], w = (R)F.c[4 * i + 2];
            s += (R)F.c[4 * i + 3] * exp(-(dx * dx + dy * dy) / (R(2) * w * w));
        }
        return s;
    }
    case DG_QPOINTS: return (R)F.vals[pidx];
    }
    return R(0);
}

// eps, b and alpha are affine in (x, y): c0 + c1 x + c2 y (constants have c1 = c2 = 0)
template <typename R>
__device__ __forceinline__ R affine_at(const FieldDev& F, R x, R y)
{
    return (R)F.c[0] + (R)F.c[1] * x + (R)F.c[2] * y;
}

template <int K, typename R>
__global__ __launch_bounds__(256) void assemble_kernel(const AsmArgs a)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, NQE = L.nqe;
    constexpr int EPW = 64 / N;  // elements per wavefront
    const R* __restrict__ tab = (const R*)a.tab;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in_wave = lane / N;
    const int j = lane - e_in_wave * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e_in_wave;
    if (e_in_wave >= EPW || el >= a.T) return;  // no barriers or cross-lane operations below

    const R cD = (a.parts & DG_PART_D) ? R(1) : R(0);
    const R cC = (a.parts & DG_PART_C) ? R(1) : R(0);
    const R cR = (a.parts & DG_PART_R) ? R(1) : R(0);
    const R kappa = (R)a.kappa;

    // ---- geometry of K (FP64, then the working precision) ----
    const double* p = a.xy + 6 * el;
    const double X1 = p[0], Y1 = p[1], X2 = p[2], Y2 = p[3], X3 = p[4], Y3 = p[5];
    const double dj11 = X2 - X1, dj12 = X3 - X1, dj21 = Y2 - Y1, dj22 = Y3 - Y1;
    const double ddet = dj11 * dj22 - dj12 * dj21;
    // G = J^{-T}: grad_x = G grad_ref
    const R G11 = (R)(dj22 / ddet), G12 = (R)(-dj21 / ddet), G21 = (R)(-dj12 / ddet), G22 = (R)(dj11 / ddet);
    const R det = (R)ddet, x1 = (R)X1, y1 = (R)Y1, j11 = (R)dj11, j12 = (R)dj12, j21 = (R)dj21, j22 = (R)dj22;

    R accd[N];
    R acco[3][N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        accd[i] = R(0);
        acco[0][i] = acco[1][i] = acco[2][i] = R(0);
    }
    // ---- volume terms ----
#pragma unroll 1
    for (int g = 0; g < NQ; ++g) {
        const R w = tab[L.vw + g] * det;
        const R xi = tab[L.vxi + g], eta = tab[L.veta + g];
        const R x = x1 + j11 * xi + j12 * eta, y = y1 + j21 * xi + j22 * eta;
        const R pj = tab[L.vphi + g * N + j], dxj = tab[L.vdx + g * N + j], dej = tab[L.vde + g * N + j];
        const R gx = G11 * dxj + G12 * dej, gy = G21 * dxj + G22 * dej;
        const R we = w * cD * affine_at<R>(a.eps, x, y);
        const R U = we * (G11 * gx + G21 * gy), V = we * (G12 * gx + G22 * gy);
        const R W = w * (cC * (affine_at<R>(a.bx, x, y) * gx + affine_at<R>(a.by, x, y) * gy) +
                         cR * affine_at<R>(a.alpha, x, y) * pj);
        const R* tp = tab + L.vphi + g * N;
        const R* tx = tab + L.vdx + g * N;
        const R* te = tab + L.vde + g * N;
#pragma unroll
        for (int i = 0; i < N; ++i) accd[i] += tx[i] * U + te[i] * V + tp[i] * W;
    }

    // ---- edge terms ----
    const int32_t nbe = a.nbr_edge[el];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const double xa = p[2 * l], ya = p[2 * l + 1];
        const double xb = p[(2 * l + 2) % 6], yb = p[(2 * l + 3) % 6];
        const double dex = xb - xa, dey = yb - ya;
        const double dlen = sqrt(dex * dex + dey * dey);
        const R len = (R)dlen, nx = (R)(dey / dlen), ny = (R)(-dex / dlen);
        const R ex = (R)dex, ey = (R)dey, xA = (R)xa, yA = (R)ya;
        const R mKx = G11 * nx + G21 * ny, mKy = G12 * nx + G22 * ny;  // G^T n
        const int32_t nb = a.nbr[3 * el + l];
        const bool interior = nb >= 0;
        const int bidx = interior ? 0 : -nb - 1;
        const bool isD = !interior && a.bnd_type[bidx] == 0;
        const bool isN = !interior && !isD;
        const R c1 = interior ? R(0.5) : (isD ? R(1) : R(0));
        const R pen = (R)((interior ? a.sigma : (isD ? a.sigma_D : 0.0)) / (a.b0 == 1.0 ? dlen : pow(dlen, a.b0)));
        R mLx = 0, mLy = 0;
        int lp = 0;
        if (interior) {
            const double* q = a.xy + 6 * (int64_t)nb;
            const double k11 = q[2] - q[0], k12 = q[4] - q[0], k21 = q[3] - q[1], k22 = q[5] - q[1];
            const double kdet = k11 * k22 - k12 * k21;
            const R H11 = (R)(k22 / kdet), H12 = (R)(-k21 / kdet), H21 = (R)(-k12 / kdet), H22 = (R)(k11 / kdet);
            mLx = H11 * nx + H21 * ny;
            mLy = H12 * nx + H22 * ny;
            lp = (nbe >> (2 * l)) & 3;
        }
        const R cI = interior ? R(1) : R(0);
#pragma unroll 1
        for (int g = 0; g < NQE; ++g) {
            const R t = tab[L.et + g];
            const R wl = tab[L.ew + g] * len;
            const R x = xA + t * ex, y = yA + t * ey;
            const R eps = affine_at<R>(a.eps, x, y);
            const R beta = affine_at<R>(a.bx, x, y) * nx + affine_at<R>(a.by, x, y) * ny;
            const R up = (!isN && beta < R(0)) ? -beta : R(0);
            const int ge = (l * NQE + g) * N;
            const R pK = tab[L.ephi + ge + j];
            const R dnK = tab[L.edx + ge + j] * mKx + tab[L.ede + ge + j] * mKy;
            const R Ad = wl * (cD * eps * (pen * pK - c1 * dnK) + cC * up * pK);
            const R Bd = wl * cD * kappa * c1 * eps * pK;
            // neighbour's trial function at the same physical point: edge lp, reversed parameter
            const int gl = (lp * NQE + (NQE - 1 - g)) * N + j;
            const R pL = cI * tab[L.ephi + gl];
            const R dnL = cI * (tab[L.edx + gl] * mLx + tab[L.ede + gl] * mLy);
            const R Ao = -wl * (cD * eps * (R(0.5) * dnL + pen * pL) + cC * up * pL);
            const R Bo = -wl * cD * kappa * R(0.5) * eps * pL;
            const R* tp = tab + L.ephi + ge;
            const R* tx = tab + L.edx + ge;
            const R* te = tab + L.ede + ge;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const R ti = tp[i];
                const R tn = tx[i] * mKx + te[i] * mKy;
                accd[i] += ti * Ad + tn * Bd;
                acco[l][i] += ti * Ao + tn * Bo;
            }
        }
    }

    // ---- atomic-free scatter through the block-row slots ----
    R* __restrict__ vals = (R*)a.vals;
    const int64_t s0 = a.row_ptr[el];
#pragma unroll
    for (int i = 0; i < N; ++i) vals[(s0 * N + i) * N + j] = accd[i];
    int slot = 1;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (a.nbr[3 * el + l] >= 0) {
            const int64_t s = s0 + slot;
#pragma unroll
            for (int i = 0; i < N; ++i) vals[(s * N + i) * N + j] = acco[l][i];
            ++slot;
        }
    }
}

// Load vector F_j = l_h(phi_j) of element K (section 1 eq. (ds)): the volume
// term f phi_j, and on boundary edges g^D ((sigma_D eps/|e|^b0 + max(-beta,0))
// phi_j + kappa eps grad phi_j . n) (Dirichlet) or g^N phi_j (Neumann).
// Lane per (element, j); kept apart from the matrix kernel so that the general
// data fields (Gaussian sums, point values) do not raise its register count.
template <int K, typename R>
__global__ __launch_bounds__(256) void load_vector_kernel(const AsmArgs a)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, NQE = L.nqe;
    constexpr int EPW = 64 / N;
    const R* __restrict__ tab = (const R*)a.tab;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in_wave = lane / N;
    const int j = lane - e_in_wave * N;
    const int64_t el = ((int64_t)blockIdx.x * 4 + wave) * EPW + e_in_wave;
    if (e_in_wave >= EPW || el >= a.T) return;

    const double* p = a.xy + 6 * el;
    const double dj11 = p[2] - p[0], dj12 = p[4] - p[0], dj21 = p[3] - p[1], dj22 = p[5] - p[1];
    const double ddet = dj11 * dj22 - dj12 * dj21;
    const R det = (R)ddet, x1 = (R)p[0], y1 = (R)p[1], j11 = (R)dj11, j12 = (R)dj12, j21 = (R)dj21, j22 = (R)dj22;
    R rhs = R(0);
#pragma unroll 1
    for (int g = 0; g < NQ; ++g) {
        const R xi = tab[L.vxi + g], eta = tab[L.veta + g];
        const R x = x1 + j11 * xi + j12 * eta, y = y1 + j21 * xi + j22 * eta;
        rhs += tab[L.vw + g] * det * field_at<R>(a.f, x, y, el * NQ + g) * tab[L.vphi + g * N + j];
    }
    const R G11 = (R)(dj22 / ddet), G12 = (R)(-dj21 / ddet), G21 = (R)(-dj12 / ddet), G22 = (R)(dj11 / ddet);
    const R kappa = (R)a.kappa;
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const int32_t nb = a.nbr[3 * el + l];
        if (nb >= 0) continue;
        const int bidx = -nb - 1;
        const bool isD = a.bnd_type[bidx] == 0;
        const double xa = p[2 * l], ya = p[2 * l + 1];
        const double xb = p[(2 * l + 2) % 6], yb = p[(2 * l + 3) % 6];
        const double dex = xb - xa, dey = yb - ya;
        const double dlen = sqrt(dex * dex + dey * dey);
        const R len = (R)dlen, nx = (R)(dey / dlen), ny = (R)(-dex / dlen);
        const R mKx = G11 * nx + G21 * ny, mKy = G12 * nx + G22 * ny;
        const R pen = (R)(a.sigma_D / (a.b0 == 1.0 ? dlen : pow(dlen, a.b0)));
#pragma unroll 1
        for (int g = 0; g < NQE; ++g) {
            const R t = tab[L.et + g];
            const R wl = tab[L.ew + g] * len;
            const R x = (R)xa + t * (R)dex, y = (R)ya + t * (R)dey;
            const int ge = (l * NQE + g) * N + j;
            const R pK = tab[L.ephi + ge];
            if (isD) {
                const R eps = affine_at<R>(a.eps, x, y);
                const R beta = affine_at<R>(a.bx, x, y) * nx + affine_at<R>(a.by, x, y) * ny;
                const R up = beta < R(0) ? -beta : R(0);
                const R dnK = tab[L.edx + ge] * mKx + tab[L.ede + ge] * mKy;
                const R gd = field_at<R>(a.gD, x, y, (int64_t)bidx * NQE + g);
                rhs += wl * gd * ((eps * pen + up) * pK + kappa * eps * dnK);
            } else {
                rhs += wl * field_at<R>(a.gN, x, y, (int64_t)bidx * NQE + g) * pK;
            }
        }
    }
    ((R*)a.rhs)[el * N + j] = rhs;
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
