// Per-element assembly device functions of the interior penalty DG system on
// gfx950, shared by the single-mesh kernels and the batched persistent kernel.
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
// Thread mapping: one lane per (element K, trial function j).  Each lane accumulates column j of the
// diagonal block and of the three neighbour blocks in registers.  The loops
// run over quadrature points g and test functions i with wave-uniform
// indices, so the test-function table values are scalar loads, while the
// per-lane work is the trial function's data at g.  Column j of each block is
// written by lane j: the n_loc lanes of an element write contiguous rows.
#pragma once

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

// Block row `el` of the matrix, column j of each block (one lane).
template <int K, typename R>
__device__ __forceinline__ void assemble_element(const AsmArgs& a, const int64_t el, const int j, R* __restrict__ vals)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, NQE = L.nqe;
    const R* __restrict__ tab = (const R*)a.tab;

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

// Boundary-edge part of the load vector entry F_j of element K (section 1
// eq. (ds)): on Dirichlet edges g^D ((sigma_D eps/|e|^b0 + max(-beta,0))
// phi_j + kappa eps grad phi_j . n), on Neumann edges g^N phi_j.  p: the
// element's vertex coordinates, G = J^{-T}.
template <int K, typename R>
__device__ __forceinline__ R load_vector_boundary(const AsmArgs& a, const int64_t el, const int j, const double* p,
                                                  R G11, R G12, R G21, R G22)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQE = L.nqe;
    const R* __restrict__ tab = (const R*)a.tab;
    const R kappa = (R)a.kappa;
    R rhs = R(0);
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
    return rhs;
}

// Volume part sum_g w_g f(x_g) phi_j(x_g) on the reference triangle (times
// det J by the caller) for f given as a function (not point values).  w, xi,
// eta: [NQ] weights and reference coordinates; phi: [NQ][N] basis values.
template <int K, typename R>
__device__ __forceinline__ R load_vector_volume_field(const AsmArgs& a, const int j, R x1, R y1, R j11, R j12, R j21,
                                                      R j22, const R* w, const R* xi, const R* eta, const R* phi)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq;
    R s = R(0);
#pragma unroll 4
    for (int g = 0; g < NQ; ++g) {
        const R x = x1 + j11 * xi[g] + j12 * eta[g], y = y1 + j21 * xi[g] + j22 * eta[g];
        s += w[g] * field_at<R>(a.f, x, y, 0) * phi[g * N + j];
    }
    return s;
}

// Load vector F_j = l_h(phi_j) of element K (section 1 eq. (ds)): the volume
// term f phi_j plus the boundary-edge terms.  Lane per (element, j); kept apart
// from the point-quadrature matrix kernel so that the general data fields
// (Gaussian sums, point values) do not raise its register count.
template <int K, typename R>
__device__ __forceinline__ void load_vector_element(const AsmArgs& a, const int64_t el, const int j, R* __restrict__ rhs_out)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq;
    const R* __restrict__ tab = (const R*)a.tab;

    const double* p = a.xy + 6 * el;
    const double dj11 = p[2] - p[0], dj12 = p[4] - p[0], dj21 = p[3] - p[1], dj22 = p[5] - p[1];
    const double ddet = dj11 * dj22 - dj12 * dj21;
    R rhs;
    if (a.f.kind == DG_QPOINTS) {  // all point values in flight at once
        const double* fv = a.f.vals + el * NQ;
        rhs = R(0);
#pragma unroll
        for (int g = 0; g < NQ; ++g) rhs += tab[L.vw + g] * (R)fv[g] * tab[L.vphi + g * N + j];
    } else {
        rhs = load_vector_volume_field<K, R>(a, j, (R)p[0], (R)p[1], (R)dj11, (R)dj12, (R)dj21, (R)dj22, tab + L.vw,
                                             tab + L.vxi, tab + L.veta, tab + L.vphi);
    }
    rhs *= (R)ddet;
    const R G11 = (R)(dj22 / ddet), G12 = (R)(-dj21 / ddet), G21 = (R)(-dj12 / ddet), G22 = (R)(dj11 / ddet);
    rhs += load_vector_boundary<K, R>(a, el, j, p, G11, G12, G21, G22);
    rhs_out[el * N + j] = rhs;
}

}  // namespace dg
