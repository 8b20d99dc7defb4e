// Single-mesh assembly kernels (see asm_device.h for the terms computed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "asm_device.h"
#include "mfma.h"

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


// Load vector, volume term: F_j = det J sum_g w_g f(x_g) phi_j(x_g).  Lane per
// (element, j); the block's f point values (contiguous in memory) are staged
// in LDS by coalesced loads and the reference weights / basis values too, so
// the per-lane loop reads only LDS.
// Volume term of the load vector, det J sum_g w_g f(x_g) phi_j(x_g), from the
// tables sw = w[NQ], phi[NQ][N], xi[NQ], eta[NQ] (in LDS); fe: the element's
// point values of f when f is given by point values (FE = R in LDS or double
// in global memory).
template <int K, typename R, typename FE>
__device__ __forceinline__ R volume_rhs(const AsmArgs& a, const R* sw, const FE* fe, bool fpts, const double* p,
                                        int j)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq;
    const double dj11 = p[2] - p[0], dj12 = p[4] - p[0], dj21 = p[3] - p[1], dj22 = p[5] - p[1];
    const double det = dj11 * dj22 - dj12 * dj21;
    R r = R(0);
    if (fpts) {
#pragma unroll
        for (int g = 0; g < NQ; ++g) r += sw[g] * (R)fe[g] * sw[NQ + g * N + j];
    } else if (a.f.kind == DG_CONST) {
#pragma unroll
        for (int g = 0; g < NQ; ++g) r += sw[g] * sw[NQ + g * N + j];
        r *= (R)a.f.c[0];
    } else {
        r = load_vector_volume_field<K, R>(a, j, (R)p[0], (R)p[1], (R)dj11, (R)dj12, (R)dj21, (R)dj22, sw, sw + NQ * (N + 1),
                                           sw + NQ * (N + 2), sw + NQ);
    }
    return r * (R)det;
}

// The point tables of volume_rhs, staged by a workgroup.
template <int K, typename R>
__device__ __forceinline__ void stage_point_tables(const AsmArgs& a, R* sw, int nthreads)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq;
    const R* __restrict__ tab = (const R*)a.tab;
    for (int t = threadIdx.x; t < NQ; t += nthreads) {
        sw[t] = tab[L.vw + t];
        sw[NQ * (N + 1) + t] = tab[L.vxi + t];
        sw[NQ * (N + 2) + t] = tab[L.veta + t];
    }
    for (int t = threadIdx.x; t < NQ * N; t += nthreads) sw[NQ + t] = tab[L.vphi + t];
}

template <int K, typename R>
__global__ __launch_bounds__(256) void load_vector_volume_kernel(const AsmArgs a)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, EPW = 64 / N, EPB = 4 * EPW;
    __shared__ R sw[NQ * (N + 3)];  // w[NQ], phi[NQ][N], xi[NQ], eta[NQ]
    __shared__ R sf[EPB * NQ];
    const bool fpts = a.f.kind == DG_QPOINTS;
    stage_point_tables<K, R>(a, sw, 256);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in = lane / N;
    const int j = lane - e_in * N;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    if (fpts) {
        const int64_t nf = (a.T - e0 < EPB ? a.T - e0 : (int64_t)EPB) * NQ;
        const double* fv = a.f.vals + e0 * NQ;
        for (int64_t t = threadIdx.x; t < nf; t += 256) sf[t] = (R)fv[t];
    }
    __syncthreads();
    const int64_t el = e0 + wave * EPW + e_in;
    if (e_in < EPW && el < a.T)
        ((R*)a.rhs)[el * N + j] = volume_rhs<K, R, R>(a, sw, sf + (el - e0) * NQ, fpts, a.xy + 6 * el, j);
}


// Load vector, boundary-edge terms, added after the volume term: thread per
// (boundary element, j), so every entry has one writer.
template <int K, typename R>
__global__ __launch_bounds__(256) void load_vector_boundary_kernel(const AsmArgs a, const int32_t* __restrict__ belems,
                                                                   int64_t nbe)
{
    constexpr int N = (K + 1) * (K + 2) / 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nbe * N) return;
    const int64_t el = belems[t / N];
    const int j = (int)(t - (t / N) * N);
    const double* p = a.xy + 6 * el;
    const double dj11 = p[2] - p[0], dj12 = p[4] - p[0], dj21 = p[3] - p[1], dj22 = p[5] - p[1];
    const double det = dj11 * dj22 - dj12 * dj21;
    const R G11 = (R)(dj22 / det), G12 = (R)(-dj21 / det), G21 = (R)(-dj12 / det), G22 = (R)(dj11 / det);
    ((R*)a.rhs)[el * N + j] += load_vector_boundary<K, R>(a, el, j, p, G11, G12, G21, G22);
}

// Boundary-edge terms of the load vector (after its volume term).
template <int K, typename R>
static void launch_load_boundary(const dg_mesh* m, const AsmArgs& a, hipStream_t s)
{
    constexpr int N = (K + 1) * (K + 2) / 2;
    // the boundary terms of l_h are g^D (...) and g^N phi: nothing to add when both vanish
    const bool zero_data = a.gD.kind == DG_CONST && a.gD.c[0] == 0.0 && a.gN.kind == DG_CONST && a.gN.c[0] == 0.0;
    const int64_t nb = (int64_t)m->bnd_elems.size();
    if (nb > 0 && !zero_data)
        hipLaunchKernelGGL((load_vector_boundary_kernel<K, R>), dim3((unsigned)((nb * N + 255) / 256)), dim3(256), 0,
                           s, a, (const int32_t*)m->d_bnd_elems, nb);
}

template <int K, typename R>
static void launch_load_vector(const dg_mesh* m, const AsmArgs& a, hipStream_t s)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPB = 4 * (64 / N);
    const int64_t grid = (m->T + EPB - 1) / EPB;
    if (grid > 0) hipLaunchKernelGGL((load_vector_volume_kernel<K, R>), dim3((unsigned)grid), dim3(256), 0, s, a);
    launch_load_boundary<K, R>(m, a, s);
}

// Constant eps, b and alpha on affine elements: every entry of the block row
// is a linear combination of the reference tensors of TenLayout with
// coefficients from the element's geometry and the problem constants (the
// same terms as assemble_element, integrated exactly by the same rules):
//   volume  det (eps (M11 SXX + M12 SXY + M22 SYY) + (G^T b) . (CX, CY) + alpha MASS),  M = G^T G,
//   edge l  |e| ((eps pen + up) E - c1 eps m_K . (DX, DY) + kappa c1 eps m_K . (TX, TY)),
//   K -> L  -|e| ((eps pen + up) F + 1/2 eps m_L . (GX, GY) + kappa 1/2 eps m_K . (HX, HY)),
// with G = J^{-T}, m = G^T n, up = max(-b . n, 0) (b . n is constant on an
// edge, so the per-point upwind decision is one decision per edge).  The
// tensors are staged in LDS; a lane (element, trial j) reads column j.  Each
// neighbour block is stored as soon as its edge is done, so that only the
// diagonal block and one neighbour block are live in registers.
constexpr int TEN_BLOCK = 512;


// Upwind term of edge l summed point by point (an edge on which b . n changes
// sign between quadrature points): acc[i] += scale sum_g w_g max(-bl(t_g), 0)
// phi_i(l, t_g) u_j, with bl(t) = blA + t dbl (|e| b . n) and u_j the trial
// function on the same edge (diagonal block) or the neighbour's trace on its
// edge lp at the same point (parameter 1 - t).
template <int K, typename R>
__device__ void upwind_points(const AsmArgs& a, int l, int lp, int j, double blA, double dbl, double scale, R* acc,
                              bool same = false)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, Q = L.nqe;
    const R* __restrict__ tab = (const R*)a.tab;
#pragma unroll 1
    for (int g = 0; g < Q; ++g) {
        const double bl = blA + (double)tab[L.et + g] * dbl;
        if (!(bl < 0.0)) continue;
        const R* ti = tab + L.ephi + (l * Q + g) * N;
        const R u = same ? ti[j] : tab[L.ephi + (lp * Q + (Q - 1 - g)) * N + j];
        const R w = (R)(scale * (double)tab[L.ew + g] * -bl) * u;
#pragma unroll
        for (int i = 0; i < N; ++i) acc[i] += w * ti[i];
    }
}

// A wave-uniform double held in scalar registers.  Selecting per lane between
// two kernel arguments otherwise becomes one vector load from the argument
// block per lane, whose wait also covers every store issued before it.
__device__ __forceinline__ double scalar_value(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Staged tensor layout: each n x n tensor as n columns (trial function j) of
// TenCol<K,R>::np values (test function i), the column padded to whole 16-byte
// words so that a lane reads its column with ds_read_b128 (P3 in FP32: 10
// floats padded to 12, three 16-byte reads instead of five 8-byte ones).
template <int K, typename R>
struct TenCol {
    static constexpr int n = (K + 1) * (K + 2) / 2;
    static constexpr int w = 16 / (int)sizeof(R);         // R per 16-byte word
    static constexpr int np = (n + w - 1) / w * w;         // padded column
    static constexpr int ts = n * np;                     // one tensor
};

// Blocks written through LDS: with STAGED, a wave puts each block of its
// elements (column j from each lane) into its own LDS buffer and writes them
// out as whole 16-byte words, consecutive lanes on consecutive words, instead
// of one 4- or 8-byte value per lane scattered over the block rows.
template <int K, typename R>
struct StagedStores {
    static constexpr int N = (K + 1) * (K + 2) / 2, NN = N * N, EPW = 64 / N;
    static constexpr bool on = (NN * (int)sizeof(R)) % 16 == 0 && K == 2;  // P3: slower (LDS and latency bound)
    static constexpr int WORDS = on ? NN * (int)sizeof(R) / 16 : 1;  // 16-byte words per block
    static constexpr int BUF = on ? EPW * NN : 0;            // R per wave
};

template <int K, typename R>
__device__ __forceinline__ void tensor_element(const AsmArgs& a, const R* st, const R* sw, const int64_t el,
                                               const int j, R* wb = nullptr, bool valid = true, int e_in = 0)
{
    constexpr int N = (K + 1) * (K + 2) / 2, NN = N * N;
    constexpr TabLayout L(K);
    using SS = StagedStores<K, R>;
    constexpr bool STAGED = SS::on;
    constexpr int NP = TenCol<K, R>::np, TS = TenCol<K, R>::ts;  // staged column and tensor strides
    const R t_first = ((const R*)a.tab)[L.et], t_last = ((const R*)a.tab)[L.et + L.nqe - 1];
    // all global loads of the element first, so that they are in flight together;
    // the neighbours enter only through the element's own table of their
    // gradient maps on the shared edges (no gathers)
    const double* p = a.xy + 6 * el;
    const double X1 = p[0], Y1 = p[1], X2 = p[2], Y2 = p[3], X3 = p[4], Y3 = p[5];
    int32_t nb[3];
    int32_t btype[3];
    // the table is loaded with the rest, except for P3: there each edge's pair
    // is loaded at the start of the previous edge's block, ahead of its stores
    // (loads and stores share one completion counter, so a load issued after
    // the stores would wait for them), which keeps 128 VGPRs without spills
    constexpr bool HOIST = K <= 2;
    double mL[6];
#pragma unroll
    for (int l = 0; l < 3; ++l) nb[l] = a.nbr[3 * el + l];
    if constexpr (HOIST) {
#pragma unroll
        for (int v = 0; v < 6; ++v) mL[v] = a.mL[6 * el + v];
    } else {
        mL[0] = a.mL[6 * el];
        mL[1] = a.mL[6 * el + 1];
    }
    const int32_t nbe = a.nbr_edge[el];
    const int64_t s0 = a.row_ptr[el];
#pragma unroll
    for (int l = 0; l < 3; ++l) btype[l] = nb[l] >= 0 ? -1 : a.bnd_type[-nb[l] - 1];
    // The volume term of the load vector (point tables in sw), computed before
    // the matrix where registers allow: its loads of f then join the ones
    // above in flight instead of being issued after the block stores, which
    // they would wait for.  P3 computes it last and reads the coordinates
    // again rather than holding them across the matrix.
    const double xyv[6] = {X1, Y1, X2, Y2, X3, Y3};
    auto load_vector = [&]() -> R {
        constexpr int NQ = L.nq;
        const bool fpts = a.f.kind == DG_QPOINTS;
        return volume_rhs<K, R, double>(a, sw, fpts ? a.f.vals + el * NQ : nullptr, fpts, HOIST ? xyv : p, j);
    };
    R rv = R(0);
    if constexpr (HOIST) {
        if (a.rhs) rv = load_vector();
    }

    const double sigma_int = scalar_value(a.sigma), sigma_dir = scalar_value(a.sigma_D);
    const double cD = (a.parts & DG_PART_D) ? 1.0 : 0.0;
    const double cC = (a.parts & DG_PART_C) ? 1.0 : 0.0;
    const double cR = (a.parts & DG_PART_R) ? 1.0 : 0.0;
    const double deps = cD * a.eps.c[0];
    // b = (bx, by), each affine: c0 + c1 x + c2 y
    const double bx1 = a.bx.c[1], bx2 = a.bx.c[2], by1 = a.by.c[1], by2 = a.by.c[2];
    const bool baff = bx1 != 0.0 || bx2 != 0.0 || by1 != 0.0 || by2 != 0.0;
    const double dj11 = X2 - X1, dj12 = X3 - X1, dj21 = Y2 - Y1, dj22 = Y3 - Y1;
    const double det = dj11 * dj22 - dj12 * dj21;
    const double inv = 1.0 / det;
    // G = J^{-T} = [[G11, G12], [G21, G22]]
    const double G11 = dj22 * inv, G12 = -dj21 * inv, G21 = -dj12 * inv, G22 = dj11 * inv;
    const R* col = st + j * NP;
    R* __restrict__ vals = (R*)a.vals;
    // edge vectors from vertex l to vertex l+1
    const double evx[3] = {dj11, dj12 - dj11, -dj12}, evy[3] = {dj21, dj22 - dj21, -dj22};

    // What edge l contributes to both its diagonal and off-diagonal terms.
    // |e| n = (dy, -dx): every edge coefficient carries the factor |e| of ds.
    // |e| b . n is linear along the edge: blA at vertex l, blA + dbl at vertex
    // l+1.  Upwinding is decided at the quadrature points; when all of them have
    // the same sign of b . n, the upwind weight max(-b . n, 0) is linear in t and
    // integrates exactly through E (and t E); otherwise (mixed) the upwind term
    // of the edge is summed point by point.
    struct EdgeCoef {
        double mKx, mKy;  // |e| G^T n
        double s, s1;     // penalty + inflow weight at vertex l, and its slope along the edge
        double blA, dbl;
        bool mixed;
    };
    auto edge_coef = [&](int l) {
        EdgeCoef e;
        const double nx = evy[l], ny = -evx[l];
        e.mKx = G11 * nx + G21 * ny;
        e.mKy = G12 * nx + G22 * ny;
        const double sig = nb[l] >= 0 ? sigma_int : sigma_dir;
        // |e| * sigma / |e|^b0
        const double pl = a.b0 == 1.0 ? sig : sig * pow(sqrt(nx * nx + ny * ny), 1.0 - a.b0);
        const double xa = l == 0 ? X1 : (l == 1 ? X2 : X3), ya = l == 0 ? Y1 : (l == 1 ? Y2 : Y3);
        e.blA = (a.bx.c[0] + bx1 * xa + bx2 * ya) * nx + (a.by.c[0] + by1 * xa + by2 * ya) * ny;
        e.dbl = (bx1 * evx[l] + bx2 * evy[l]) * nx + (by1 * evx[l] + by2 * evy[l]) * ny;
        const double bl0 = e.blA + (double)t_first * e.dbl, bl1 = e.blA + (double)t_last * e.dbl;
        const bool inflow = bl0 < 0.0 && bl1 < 0.0;
        e.mixed = (bl0 < 0.0) != (bl1 < 0.0);
        e.s = deps * pl + cC * (inflow ? -e.blA : 0.0);
        e.s1 = cC * (inflow ? -e.dbl : 0.0);
        return e;
    };

    // STAGED: every lane of the wave calls this for the same block (slot < 0
    // where the lane's element has no such block or is not a real element)
    auto put_block = [&](const R* acc, int32_t slot_l) {
        const int lane = (int)(threadIdx.x & 63);
        if (slot_l >= 0) {
#pragma unroll
            for (int i = 0; i < N; ++i) wb[e_in * NN + i * N + j] = acc[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        constexpr int TOT = SS::EPW * SS::WORDS, IT = (TOT + 63) / 64;
        int32_t se[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {  // every lane active: slot of the element of word lane + 64 it
            const int c = lane + 64 * it;
            const int e = (c < TOT ? c : TOT - 1) / SS::WORDS;
            se[it] = __shfl(slot_l, e * N, 64);
        }
        R* __restrict__ vals = (R*)a.vals;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int c = lane + 64 * it;
            if (c < TOT && se[it] >= 0) {
                const int e = c / SS::WORDS, w = c - e * SS::WORDS;
                const uint4 v = reinterpret_cast<const uint4*>(wb + e * NN)[w];
                reinterpret_cast<uint4*>(vals + (int64_t)se[it] * NN)[w] = v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };

    // Off-diagonal block of interior edge l (into acco).
    int64_t slot = s0 + 1;
    auto off_block = [&](int l, const EdgeCoef& e, R* acco) {
        const double hk = 0.5 * deps;
        const int lp = (nbe >> (2 * l)) & 3;
        R c[5];
        c[0] = (R)(-e.s);
        c[1] = (R)(-hk * mL[2 * l]);  // -1/2 eps |e| m_L
        c[2] = (R)(-hk * mL[2 * l + 1]);
        c[3] = (R)(-0.5 * deps * a.kappa * e.mKx);
        c[4] = (R)(-0.5 * deps * a.kappa * e.mKy);
        const R* Tl = col + (TenStage::EO + 5 * (3 * l + lp)) * TS;
#pragma unroll
        for (int i = 0; i < N; ++i) acco[i] = c[0] * Tl[i];
#pragma unroll
        for (int t = 1; t < 5; ++t) {
            const R* T = Tl + t * TS;
#pragma unroll
            for (int i = 0; i < N; ++i) acco[i] += c[t] * T[i];
        }
        if (baff) {
            const R c1t = (R)(-e.s1);
            const R* T1 = col + (TenStage::F1 + 3 * l + lp) * TS;
#pragma unroll
            for (int i = 0; i < N; ++i) acco[i] += c1t * T1[i];
            if (e.mixed) upwind_points<K, R>(a, l, lp, j, e.blA, e.dbl, -cC, acco);
        }
    };
    // ... stored as soon as it is complete
    auto off_diagonal = [&](int l, const EdgeCoef& e) {
        R acco[N];
        off_block(l, e, acco);
#pragma unroll
        for (int i = 0; i < N; ++i) vals[(slot * N + i) * N + j] = acco[i];
        ++slot;
    };
    // The off-diagonal blocks first, then the diagonal block: their stores
    // drain while the diagonal block is summed, and the two sets of
    // accumulators are never live together.  Each block sums its terms in the
    // same order as one pass over the edges would.
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if constexpr (!HOIST) {
            if (l < 2) {
                mL[2 * l + 2] = a.mL[6 * el + 2 * l + 2];
                mL[2 * l + 3] = a.mL[6 * el + 2 * l + 3];
            }
        }
        if constexpr (STAGED) {  // every lane takes part in every edge's block write
            R acco[N];
#pragma unroll
            for (int i = 0; i < N; ++i) acco[i] = R(0);
            const bool has = nb[l] >= 0;
            if (has) off_block(l, edge_coef(l), acco);
            put_block(acco, valid && has ? (int32_t)slot : -1);
            if (has) ++slot;
        } else if (nb[l] >= 0) {
            off_diagonal(l, edge_coef(l));
        }
    }

    R accd[N];
#pragma unroll
    for (int i = 0; i < N; ++i) accd[i] = R(0);
    {
        // det (G^T G) = adj(J)^T adj(J) / det
        const double ed = deps * inv;
        R c[6];
        c[0] = (R)(ed * (dj22 * dj22 + dj12 * dj12));
        c[1] = (R)(-ed * (dj22 * dj21 + dj12 * dj11));
        c[2] = (R)(ed * (dj21 * dj21 + dj11 * dj11));
        // det G^T b(xi, eta), b at vertex 1 plus its slopes along xi and eta
        const double bx0 = a.bx.c[0] + bx1 * X1 + bx2 * Y1, by0 = a.by.c[0] + by1 * X1 + by2 * Y1;
        c[3] = (R)(cC * (dj22 * bx0 - dj12 * by0));
        c[4] = (R)(cC * (dj11 * by0 - dj21 * bx0));
        c[5] = (R)(cR * a.alpha.c[0] * det);
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const R* T = col + (TenStage::VOL + t) * TS;
#pragma unroll
            for (int i = 0; i < N; ++i) accd[i] += c[t] * T[i];
        }
        if (baff) {
            const double bxa = bx1 * dj11 + bx2 * dj21, bxb = bx1 * dj12 + bx2 * dj22;  // d bx / d xi, d eta
            const double bya = by1 * dj11 + by2 * dj21, byb = by1 * dj12 + by2 * dj22;
            R cb[4];
            cb[0] = (R)(cC * (dj22 * bxa - dj12 * bya));
            cb[1] = (R)(cC * (dj22 * bxb - dj12 * byb));
            cb[2] = (R)(cC * (dj11 * bya - dj21 * bxa));
            cb[3] = (R)(cC * (dj11 * byb - dj21 * bxb));
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const R* T = col + (TenStage::VB + t) * TS;
#pragma unroll
                for (int i = 0; i < N; ++i) accd[i] += cb[t] * T[i];
            }
        }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (btype[l] == 1) continue;  // Neumann edge: load vector only
        const EdgeCoef e = edge_coef(l);
        const double dc = deps * (nb[l] >= 0 ? 0.5 : 1.0);
        const R c0 = (R)e.s, cx = (R)(dc * e.mKx), cy = (R)(dc * e.mKy);
        const R* T = col + (TenStage::ED + 3 * l) * TS;
#pragma unroll
        for (int i = 0; i < N; ++i) accd[i] += c0 * T[i] + cx * T[TS + i] + cy * T[2 * TS + i];
        if (baff) {
            const R c1t = (R)e.s1;
            const R* T1 = col + (TenStage::E1 + l) * TS;
#pragma unroll
            for (int i = 0; i < N; ++i) accd[i] += c1t * T1[i];
        }
        if (baff && e.mixed) upwind_points<K, R>(a, l, l, j, e.blA, e.dbl, cC, accd, true);
    }
    if constexpr (STAGED) {
        put_block(accd, valid ? (int32_t)s0 : -1);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) vals[(s0 * N + i) * N + j] = accd[i];
    }
    if (a.rhs) {
        if constexpr (!HOIST) rv = load_vector();
        if (valid) ((R*)a.rhs)[el * N + j] = rv;
    }
}


template <int K, typename R>
__global__ __launch_bounds__(TEN_BLOCK, 4) void assemble_tensor_kernel(const AsmArgs a, const R* __restrict__ ten)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NN = N * N, NQ = L.nq, EPW = 64 / N, WPB = TEN_BLOCK / 64;
    constexpr int NT = TenStage::COUNT * TenCol<K, R>::ts;
    constexpr int RPW = 16 / (int)sizeof(R);
    constexpr int PER = (NT / RPW + TEN_BLOCK - 1) / TEN_BLOCK;  // 16-byte tensor words per thread
    constexpr int NTP = PER * TEN_BLOCK * RPW;                   // tensor region padded to whole passes
    constexpr int SWP = (NQ * (N + 3) + RPW - 1) / RPW * RPW;    // point tables padded to whole words
    using SS = StagedStores<K, R>;
    // staged tensors, the load vector's point tables, then (STAGED) each wave's block buffer
    __shared__ __align__(16) R st[NTP + SWP + WPB * SS::BUF];
    R* sw = st + NTP;
    const bool baff = a.bx.c[1] != 0.0 || a.bx.c[2] != 0.0 || a.by.c[1] != 0.0 || a.by.c[2] != 0.0;
    // Staging: every load of a thread (the tensors in 16-byte words, then the
    // load vector's point tables) is issued before its first LDS write, so the
    // workgroup waits for one round trip instead of one per word; the empty asm
    // with a memory clobber keeps the compiler from sinking loads into the
    // guarded writes.  Both staged tensor sets are whole 16-byte words and each
    // method's set starts on one (the host packs them contiguously from a
    // hipMalloc base).
    static_assert(NT % RPW == 0 && (TenStage::CONST_B * TenCol<K, R>::ts) % RPW == 0,
                  "staged tensors are whole 16-byte words");
    constexpr int PPT = (NQ * N + TEN_BLOCK - 1) / TEN_BLOCK;
    static_assert(NQ <= TEN_BLOCK, "one point per thread");
    const int nw = (baff ? TenStage::COUNT : TenStage::CONST_B) * TenCol<K, R>::ts / RPW;
    const R* __restrict__ tab = (const R*)a.tab;
    uint4 buf[PER];
    R pt[3], pphi[PPT];
    {
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(ten);
        // a word past the staged set re-reads word 0 and lands in the tensor
        // slots that a constant b leaves unread, or in the padding
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int t = threadIdx.x + p * TEN_BLOCK;
            buf[p] = src[t < nw ? t : 0];
        }
        const int q = threadIdx.x < NQ ? threadIdx.x : 0;
        pt[0] = tab[L.vw + q];
        pt[1] = tab[L.vxi + q];
        pt[2] = tab[L.veta + q];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int t = threadIdx.x + p * TEN_BLOCK;
            pphi[p] = tab[L.vphi + (t < NQ * N ? t : 0)];
        }
    }
    asm volatile("" ::: "memory");
    {
        uint4* dst = reinterpret_cast<uint4*>(st);
#pragma unroll
        for (int p = 0; p < PER; ++p) dst[threadIdx.x + p * TEN_BLOCK] = buf[p];
        // point tables (same layout as stage_point_tables): weights, basis
        // values, then the reference coordinates
        if (a.rhs) {
            const int q = threadIdx.x;
            if (q < NQ) {
                sw[q] = pt[0];
                sw[NQ * (N + 1) + q] = pt[1];
                sw[NQ * (N + 2) + q] = pt[2];
            }
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const int t = threadIdx.x + p * TEN_BLOCK;
                if (t < NQ * N) sw[NQ + t] = pphi[p];
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e_in = lane / N;
    const int j = lane - e_in * N;
    const int64_t e0 = ((int64_t)blockIdx.x * WPB + wave) * EPW;
    const int64_t el = e0 + e_in;
    if constexpr (SS::on) {
        // every lane of a wave with a real element takes part in the block writes;
        // the others compute a copy of the wave's first element and write nothing
        if (e0 >= a.T) return;
        const bool valid = e_in < EPW && el < a.T;
        tensor_element<K, R>(a, st, sw, valid ? el : e0, j, st + NTP + SWP + wave * SS::BUF, valid,
                             e_in < EPW ? e_in : 0);
    } else {
        if (e_in >= EPW || el >= a.T) return;
        tensor_element<K, R>(a, st, sw, el, j);
    }
}

// ---------------------------------------------------------------------------
// Matrix-core assembly (k = 2, 3).  Every block the tensor kernel sums is a
// combination of reference tensors with per-element coefficients, so for a
// tile of 16 elements each block type is the product C B of their 16 x K
// coefficient rows C with K tensors B laid out as rows of n^2 entries (MfmaSet).
// Two launches:
//   mf_coef_kernel        one lane per element: the element's coefficients (as
//                         rows of a coefficient array, element-minor, so that
//                         the stores coalesce) and the volume term of its load
//                         vector;
//   assemble_mfma_kernel  v_mfma_*_16x16x4 products, four tensors per step:
//                         lane (q, r) = (lane / 16, lane % 16) supplies the
//                         coefficient of tensor 4 s + q for the tile's element r
//                         and the value of that tensor at entry 16 c + r of
//                         column tile c, and receives entry 16 c + r of four of
//                         the tile's elements.
// A tensor value read from LDS then serves 16 elements instead of one, and the
// product kernel does little besides reading coefficients, multiplying and
// storing.  A wave takes 32 consecutive elements as two tiles, the even and
// the odd ones: on a structured mesh the two triangle types alternate, and
// each type has one neighbour edge lp per local edge, so a tile needs one
// neighbour tensor set per edge (other meshes take one product per lp present
// in the tile).  The coefficients of the next tile are loaded before the
// stores of the current one are issued, and every tile issues the same number
// of stores (buffer stores whose out-of-range lanes the hardware drops), so
// that a wave waits for its loads without waiting for its earlier stores (both
// share one completion counter).  Edges on which b . n changes sign add their
// upwind term point by point, as products with point tensors read from global
// memory (such edges are rare; those reads do wait for the stores before them).
// ---------------------------------------------------------------------------
constexpr int MF_BLOCK = 512;

// A byte range for buffer stores: offsets at or beyond MF_DROP are outside it
// and the hardware discards those lanes' stores.
constexpr uint32_t MF_DROP = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mf_range(void* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)(MF_DROP - 16u), 0x00020000);
}

// c[4 s + q] for the lane's q without indexing registers by a lane value
template <typename R>
__device__ __forceinline__ R pick4(int q, double c0, double c1, double c2, double c3)
{
    return (R)(q == 0 ? c0 : (q == 1 ? c1 : (q == 2 ? c2 : c3)));
}

// LDS tables of the product kernel besides the tensor sets (precision R):
// the edge parameters and weights [8] each (zero beyond the rule).
template <int K>
struct MfTables {
    static constexpr int ET = 0, EW = 8, SIZE = 16;
};

// Rows of the coefficient array (precision R, row-major [ROWS][T]).
struct MfCoef {
    static constexpr int VOL = 0;    // 10: SXX SXY SYY CX CY MASS VB0..VB3 (MfmaSet diagonal rows 0..9)
    static constexpr int EDGE = 10;  // 3 x 4: E, kappa TX - DX, kappa TY - DY, E1 of edge l (0 on Neumann edges)
    static constexpr int OFF = 22;   // 3 x 6: F, GX, GY, HX, HY, F1 of the neighbour block across edge l
    static constexpr int UPW = 40;   // 3 x 2: |e| b . n at vertex l and its change along edge l (affine b)
    static constexpr int MIX = 46;   // bit l: b . n changes sign along edge l (affine b)
    static constexpr int ROWS = 47;
};

// Coefficients and the volume term of the load vector, one lane per element.
// BAFF: b affine (else constant); FK: f constant (0), point values (1),
// evaluated at the volume points (2).
template <int K, typename R, bool BAFF, int FK>
__global__ __launch_bounds__(256) void mf_coef_kernel(const AsmArgs a, const int32_t* __restrict__ ebits,
                                                      R* __restrict__ coef)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NQ = L.nq, Q = L.nqe;
    __shared__ R sw[NQ * (N + 3)];  // w[NQ], phi[NQ][N], xi[NQ], eta[NQ] (stage_point_tables)
    if (a.rhs) stage_point_tables<K, R>(a, sw, 256);
    __syncthreads();
    const int64_t el = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (el >= a.T) return;
    const int64_t T = a.T;
    const R* __restrict__ tab = (const R*)a.tab;
    const double* p = a.xy + 6 * el;
    const double X1 = p[0], Y1 = p[1], X2 = p[2], Y2 = p[3], X3 = p[4], Y3 = p[5];
    const double* pm = a.mL + 6 * el;
    const int32_t bits = ebits[el];

    const double cD = (a.parts & DG_PART_D) ? 1.0 : 0.0;
    const double cC = (a.parts & DG_PART_C) ? 1.0 : 0.0;
    const double cR = (a.parts & DG_PART_R) ? 1.0 : 0.0;
    const double deps = cD * a.eps.c[0];
    const double bx1 = a.bx.c[1], bx2 = a.bx.c[2], by1 = a.by.c[1], by2 = a.by.c[2];
    const double dj11 = X2 - X1, dj12 = X3 - X1, dj21 = Y2 - Y1, dj22 = Y3 - Y1;
    const double det = dj11 * dj22 - dj12 * dj21;
    const double inv = 1.0 / det;
    const double G11 = dj22 * inv, G12 = -dj21 * inv, G21 = -dj12 * inv, G22 = dj11 * inv;
    const double t_first = (double)tab[L.et], t_last = (double)tab[L.et + Q - 1];
    auto put = [&](int row, double v) { coef[row * T + el] = (R)v; };

    // volume terms (same coefficients as tensor_element)
    {
        const double ed = deps * inv;
        const double bx0 = a.bx.c[0] + bx1 * X1 + bx2 * Y1, by0 = a.by.c[0] + by1 * X1 + by2 * Y1;
        const double bxa = bx1 * dj11 + bx2 * dj21, bxb = bx1 * dj12 + bx2 * dj22;  // d bx / d xi, d eta
        const double bya = by1 * dj11 + by2 * dj21, byb = by1 * dj12 + by2 * dj22;
        put(MfCoef::VOL + 0, ed * (dj22 * dj22 + dj12 * dj12));
        put(MfCoef::VOL + 1, -ed * (dj22 * dj21 + dj12 * dj11));
        put(MfCoef::VOL + 2, ed * (dj21 * dj21 + dj11 * dj11));
        put(MfCoef::VOL + 3, cC * (dj22 * bx0 - dj12 * by0));
        put(MfCoef::VOL + 4, cC * (dj11 * by0 - dj21 * bx0));
        put(MfCoef::VOL + 5, cR * a.alpha.c[0] * det);
        put(MfCoef::VOL + 6, cC * (dj22 * bxa - dj12 * bya));
        put(MfCoef::VOL + 7, cC * (dj22 * bxb - dj12 * byb));
        put(MfCoef::VOL + 8, cC * (dj11 * bya - dj21 * bxa));
        put(MfCoef::VOL + 9, cC * (dj11 * byb - dj21 * bxb));
    }
    // edges: |e| n = (dy, -dx) along the edge from vertex l to vertex l+1
    const double evx[3] = {dj11, dj12 - dj11, -dj12}, evy[3] = {dj21, dj22 - dj21, -dj22};
    const double vx[3] = {X1, X2, X3}, vy[3] = {Y1, Y2, Y3};
    int32_t mix = 0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const bool has = ((bits >> (8 + l)) & 1) != 0, neu = ((bits >> (12 + l)) & 1) != 0;
        const double nx = evy[l], ny = -evx[l];
        const double mKx = G11 * nx + G21 * ny, mKy = G12 * nx + G22 * ny;
        const double sig = has ? a.sigma : a.sigma_D;
        const double pl = a.b0 == 1.0 ? sig : sig * pow(sqrt(nx * nx + ny * ny), 1.0 - a.b0);
        const double blA = (a.bx.c[0] + bx1 * vx[l] + bx2 * vy[l]) * nx + (a.by.c[0] + by1 * vx[l] + by2 * vy[l]) * ny;
        const double dbl = (bx1 * evx[l] + bx2 * evy[l]) * nx + (by1 * evx[l] + by2 * evy[l]) * ny;
        const double bl0 = blA + t_first * dbl, bl1 = blA + t_last * dbl;
        const bool inflow = bl0 < 0.0 && bl1 < 0.0;
        const bool mixed = (bl0 < 0.0) != (bl1 < 0.0);
        const double es = deps * pl + cC * (inflow ? -blA : 0.0);
        const double es1 = cC * (inflow ? -dbl : 0.0);
        const double dc = deps * (has ? 0.5 : 1.0);
        put(MfCoef::EDGE + 4 * l, neu ? 0.0 : es);
        put(MfCoef::EDGE + 4 * l + 1, neu ? 0.0 : dc * mKx);
        put(MfCoef::EDGE + 4 * l + 2, neu ? 0.0 : dc * mKy);
        put(MfCoef::EDGE + 4 * l + 3, neu ? 0.0 : es1);
        const double hk = 0.5 * deps, hkk = 0.5 * deps * a.kappa;
        put(MfCoef::OFF + 6 * l, has ? -es : 0.0);
        put(MfCoef::OFF + 6 * l + 1, has ? -hk * pm[2 * l] : 0.0);
        put(MfCoef::OFF + 6 * l + 2, has ? -hk * pm[2 * l + 1] : 0.0);
        put(MfCoef::OFF + 6 * l + 3, has ? -hkk * mKx : 0.0);
        put(MfCoef::OFF + 6 * l + 4, has ? -hkk * mKy : 0.0);
        put(MfCoef::OFF + 6 * l + 5, has ? -es1 : 0.0);
        if constexpr (BAFF) {
            coef[(MfCoef::UPW + 2 * l) * T + el] = (R)blA;
            coef[(MfCoef::UPW + 2 * l + 1) * T + el] = (R)dbl;
            if (mixed) mix |= 1 << l;
        }
    }
    if constexpr (BAFF) coef[MfCoef::MIX * T + el] = (R)mix;

    // volume term of the load vector: det sum_g w_g f(x_g) phi_j(x_g)
    if (a.rhs) {
        double rj[N];
#pragma unroll
        for (int j = 0; j < N; ++j) rj[j] = 0.0;
        const double* fe = a.f.vals + el * NQ;
#pragma unroll 1
        for (int g = 0; g < NQ; ++g) {
            double fg;
            if constexpr (FK == 1) {
                fg = fe[g];
            } else if constexpr (FK == 0) {
                fg = a.f.c[0];
            } else {
                const double xi = (double)sw[NQ * (N + 1) + g], eta = (double)sw[NQ * (N + 2) + g];
                fg = field_at<double>(a.f, X1 + dj11 * xi + dj12 * eta, Y1 + dj21 * xi + dj22 * eta, 0);
            }
            const double wf = (double)sw[g] * fg;
#pragma unroll
            for (int j = 0; j < N; ++j) rj[j] += wf * (double)sw[NQ + g * N + j];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) ((R*)a.rhs)[el * N + j] = (R)(rj[j] * det);
    }
}

// The coefficients a lane reads for its row's element (one tile ahead): the
// one of each step that it supplies, the block row's first slot and the bits.
struct MfRowA {
    double vol[3];            // steps of the volume tensors (the third: affine b)
    double edge[3];           // diagonal step of edge l
    double off0[3], off1[3];  // the two steps of edge l's neighbour block
    int32_t bits, s0, mix;
};

template <typename R, bool BAFF>
__device__ __forceinline__ void mf_load_row(const R* __restrict__ coef, const int32_t* __restrict__ ebits,
                                            const int32_t* __restrict__ row_ptr, const int64_t T, const int64_t el,
                                            const int q, MfRowA& d)
{
    auto at = [&](int row) { return (double)coef[row * T + el]; };
    const int q2 = q < 2 ? q : 0;  // rows 4 s + q past the end of a set read row 0 and supply zero
    d.vol[0] = at(MfCoef::VOL + q);
    d.vol[1] = at(MfCoef::VOL + 4 + q);
    d.vol[2] = BAFF ? at(MfCoef::VOL + 8 + q2) : 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        d.edge[l] = at(MfCoef::EDGE + 4 * l + q);
        d.off0[l] = at(MfCoef::OFF + 6 * l + q);
        d.off1[l] = at(MfCoef::OFF + 6 * l + 4 + q2);
    }
    d.bits = ebits[el];
    d.s0 = row_ptr[el];
    d.mix = BAFF ? (int32_t)at(MfCoef::MIX) : 0;
    if (q >= 2) {
        d.vol[2] = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) d.off1[l] = 0.0;
    }
}

// One tile of 16 elements: rows r are the elements e_first + 2 r (those at or
// beyond T are copies of element T - 1 and store nothing); el is row r's
// element (clamped).
template <int K, typename R, bool BAFF>
__device__ __forceinline__ void mf_tile(const AsmArgs& a, const R* st, const R* tb, const R* __restrict__ tp,
                                        const R* __restrict__ coef, const MfRowA& d, const int64_t el,
                                        const int64_t e_first, const int q, const int r)
{
    constexpr TabLayout L(K);
    constexpr int N = L.n, NN = N * N, Q = L.nqe;
    constexpr int NNP = MfmaSet::nnp(K), CT = NNP / 16;
    static_assert(Q <= MfmaSet::PTS && MfmaSet::PTS == 8, "two steps of point tensors per edge");
    using Op = MfmaOp<R>;
    using V = typename Op::V;
    const int32_t bits = d.bits;
    const double cC = (a.parts & DG_PART_C) ? 1.0 : 0.0;

    V acc[CT];
    auto clear = [&]() {
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = V{0, 0, 0, 0};
    };
    // one step of four tensors; B points at this lane's tensor row 4 s + q
    auto step = [&](R av, const R* B) {
        R b[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) b[c] = B[16 * c + r];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = Op::mac(av, b[c], acc[c]);
    };
    // the block of each row at its slot (slot < 0: none); a fixed number of stores
    const int32_t sbase = __builtin_amdgcn_readfirstlane(d.s0);
    const __amdgpu_buffer_rsrc_t rv = mf_range((R*)a.vals + (int64_t)sbase * NN);
    auto store = [&](int32_t slot) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t sl = __shfl(slot, Op::row(q, i), 64);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const bool ok = sl >= 0 && 16 * c + r < NN;
                Op::store(acc[c][i], rv, ok ? (uint32_t)(((sl - sbase) * NN + 16 * c + r) * (int)sizeof(R)) : MF_DROP);
            }
        }
    };
    // point-by-point upwind term of edge l (rows whose edge l is mixed): weight
    // of point g = 4 s + q, scaled by cC on the diagonal and -cC across the edge
    auto point_coef = [&](int l, int s, double scale) -> R {
        const int g = 4 * s + q;
        const int64_t T = a.T;
        const double blA = (double)coef[(MfCoef::UPW + 2 * l) * T + el];
        const double dbl = (double)coef[(MfCoef::UPW + 2 * l + 1) * T + el];
        const double bl = blA + (double)tb[MfTables<K>::ET + g] * dbl;
        return (g < Q && bl < 0.0) ? (R)(scale * (double)tb[MfTables<K>::EW + g] * -bl) : R(0);
    };
    const bool valid = e_first + 2 * r < a.T;

    // diagonal block: volume tensors (two steps, a third for affine b), then one step per edge
    clear();
    step((R)d.vol[0], st + q * NNP);
    step((R)d.vol[1], st + (4 + q) * NNP);
    if constexpr (BAFF) step((R)d.vol[2], st + (8 + q) * NNP);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        step((R)d.edge[l], st + (12 + 4 * l + q) * NNP);
        if constexpr (BAFF) {
            const bool mx = ((d.mix >> l) & 1) && !((bits >> (12 + l)) & 1);
            if (__any(mx)) {
                step(mx ? point_coef(l, 0, cC) : R(0), tp + (l * MfmaSet::PTS + q) * NNP);
                step(mx ? point_coef(l, 1, cC) : R(0), tp + (l * MfmaSet::PTS + 4 + q) * NNP);
            }
        }
    }
    store(valid ? d.s0 : -1);

    // neighbour blocks, in the order of the block row (edges with a neighbour)
    int32_t slot = d.s0 + 1;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const bool hl = ((bits >> (8 + l)) & 1) != 0;
        const int lp = hl ? (bits >> (2 * l)) & 3 : -1;
        const int32_t my_slot = valid && hl ? slot : -1;
        if (hl) ++slot;
        clear();
#pragma unroll 1
        for (int lq = 0; lq < 3; ++lq) {
            const bool mine = lp == lq;
            if (!__any(mine)) continue;
            const R* B = st + (MfmaSet::DIAG + MfmaSet::OFF * (3 * l + lq) + q) * NNP;
            step(mine ? (R)d.off0[l] : R(0), B);
            step(mine ? (R)d.off1[l] : R(0), B + 4 * NNP);
            if constexpr (BAFF) {
                const bool mx = mine && ((d.mix >> l) & 1);
                if (__any(mx)) {
                    const R* P = tp + ((3 + 3 * l + lq) * MfmaSet::PTS + q) * NNP;
                    step(mx ? point_coef(l, 0, -cC) : R(0), P);
                    step(mx ? point_coef(l, 1, -cC) : R(0), P + 4 * NNP);
                }
            }
        }
        store(my_slot);
    }
}

template <int K, typename R, bool BAFF>
__global__ __launch_bounds__(MF_BLOCK) void assemble_mfma_kernel(const AsmArgs a, const int32_t* __restrict__ ebits,
                                                                 const R* __restrict__ tm, const R* __restrict__ tp,
                                                                 const R* __restrict__ coef)
{
    constexpr TabLayout L(K);
    constexpr int Q = L.nqe, WPB = MF_BLOCK / 64;
    using TB = MfTables<K>;
    constexpr int NT = MfmaSet::COUNT * MfmaSet::nnp(K);
    constexpr int RPW = 16 / (int)sizeof(R);
    static_assert(NT % RPW == 0, "tensor sets are whole 16-byte words");
    __shared__ __align__(16) R st[NT + TB::SIZE];
    R* tb = st + NT;
    {
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(tm);
        uint4* dst = reinterpret_cast<uint4*>(st);
        for (int t = threadIdx.x; t < NT / RPW; t += MF_BLOCK) dst[t] = src[t];
        const R* __restrict__ tab = (const R*)a.tab;
        for (int t = threadIdx.x; t < 8; t += MF_BLOCK) {
            tb[TB::ET + t] = t < Q ? tab[L.et + t] : R(0);
            tb[TB::EW + t] = t < Q ? tab[L.ew + t] : R(0);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
    const int64_t nwt = (a.T + 31) / 32;  // wave tiles of 32 elements, two tiles each
    const int64_t stride = (int64_t)gridDim.x * WPB;
    const int64_t w0 = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    if (w0 >= nwt) return;
    auto elem = [&](int64_t wt, int par) {
        const int64_t e = wt * 32 + 2 * r + par;
        return e < a.T ? e : a.T - 1;
    };
    MfRowA cur;
    int64_t ecur = elem(w0, 0);
    mf_load_row<R, BAFF>(coef, ebits, a.row_ptr, a.T, ecur, q, cur);
    for (int64_t pass = 0;; ++pass) {
        const int par = (int)(pass & 1);
        const int64_t wt = w0 + (pass >> 1) * stride;
        const int64_t wn = par ? wt + stride : wt;  // the next tile: the odd half, or the next wave tile
        const bool more = wn < nwt;
        const int64_t enext = more ? elem(wn, par ^ 1) : a.T - 1;
        MfRowA nxt;
        mf_load_row<R, BAFF>(coef, ebits, a.row_ptr, a.T, enext, q, nxt);
        mf_tile<K, R, BAFF>(a, st, tb, tp, coef, cur, ecur, wt * 32 + par, q, r);
        if (!more) break;
        cur = nxt;
        ecur = enext;
    }
}

template <int K, typename R, bool BAFF, int FK>
static void launch_mfma_v(const dg_mesh* m, const AsmArgs& a, const R* tm, const R* tp, hipStream_t s)
{
    static int per_cu = 0, cus = 0;
    if (per_cu == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, assemble_mfma_kernel<K, R, BAFF>, MF_BLOCK, 0);
        if (per_cu < 1) per_cu = 1;
        if (cus < 1) cus = 1;
    }
    R* coef = (R*)m->d_mfcoef;
    hipLaunchKernelGGL((mf_coef_kernel<K, R, BAFF, FK>), dim3((unsigned)((m->T + 255) / 256)), dim3(256), 0, s, a,
                       m->d_ebits, coef);
    const int64_t nwt = (m->T + 31) / 32;
    const int64_t want = (nwt + MF_BLOCK / 64 - 1) / (MF_BLOCK / 64);
    const int64_t grid = std::min<int64_t>(want, (int64_t)per_cu * cus);
    hipLaunchKernelGGL((assemble_mfma_kernel<K, R, BAFF>), dim3((unsigned)grid), dim3(MF_BLOCK), 0, s, a,
                       m->d_ebits, tm, tp, (const R*)coef);
}

template <int K, typename R>
static void launch_mfma(const dg_mesh* m, const AsmArgs& a, const R* tm, const R* tp, hipStream_t s)
{
    const bool baff = a.bx.c[1] != 0.0 || a.bx.c[2] != 0.0 || a.by.c[1] != 0.0 || a.by.c[2] != 0.0;
    const int fk = a.f.kind == DG_CONST ? 0 : (a.f.kind == DG_QPOINTS ? 1 : 2);
    if (baff) {
        if (fk == 0) launch_mfma_v<K, R, true, 0>(m, a, tm, tp, s);
        else if (fk == 1) launch_mfma_v<K, R, true, 1>(m, a, tm, tp, s);
        else launch_mfma_v<K, R, true, 2>(m, a, tm, tp, s);
    } else {
        if (fk == 0) launch_mfma_v<K, R, false, 0>(m, a, tm, tp, s);
        else if (fk == 1) launch_mfma_v<K, R, false, 1>(m, a, tm, tp, s);
        else launch_mfma_v<K, R, false, 2>(m, a, tm, tp, s);
    }
}

// eps and alpha constant (the affine form with zero slopes), b affine
static bool constant_coefficients(const AsmArgs& a)
{
    const FieldDev* f[2] = {&a.eps, &a.alpha};
    for (const FieldDev* F : f)
        if (F->c[1] != 0.0 || F->c[2] != 0.0) return false;
    return true;
}

template <int K, typename R>
static int launch_k(const dg_mesh* m, const AsmArgs& a, hipStream_t s)
{
    constexpr int N = (K + 1) * (K + 2) / 2, EPW = 64 / N;
    const int64_t per_block = 4 * EPW;
    const int64_t blocks = (m->T + per_block - 1) / per_block;
    if (blocks <= 0) return DG_OK;
    bool done = false;
    if constexpr (K <= 3) {
        const R* ten = std::is_same<R, double>::value ? (const R*)(const void*)m->d_ten64
                                                      : (const R*)(const void*)m->d_ten32;
        // the staged sets of this method (kappa = -1, 0, 1)
        const int ki = a.kappa < 0 ? 0 : (a.kappa > 0 ? 2 : 1);
        if constexpr (K >= 2) {
            const R* tm = std::is_same<R, double>::value ? (const R*)(const void*)m->d_tm64
                                                         : (const R*)(const void*)m->d_tm32;
            const R* tp = std::is_same<R, double>::value ? (const R*)(const void*)m->d_tp64
                                                         : (const R*)(const void*)m->d_tp32;
            if (a.vals && tm && tp && constant_coefficients(a) && (a.parts & DG_ASM_MATRIX_CORE)) {
                if (!m->d_mfcoef &&
                    hipMalloc(&m->d_mfcoef, (size_t)MfCoef::ROWS * std::max<int64_t>(m->T, 1) * sizeof(double)) !=
                        hipSuccess) {
                    m->d_mfcoef = nullptr;
                    return DG_ERR_OOM;
                }
                launch_mfma<K, R>(m, a, tm + (size_t)ki * MfmaSet::COUNT * MfmaSet::nnp(K), tp, s);
                if (a.rhs) launch_load_boundary<K, R>(m, a, s);
                done = true;
            }
        }
        if (!done && a.vals && ten && constant_coefficients(a)) {
            const int64_t per = (TEN_BLOCK / 64) * EPW;
            const int64_t grid = (m->T + per - 1) / per;
            hipLaunchKernelGGL((assemble_tensor_kernel<K, R>), dim3((unsigned)grid), dim3(TEN_BLOCK), 0, s, a,
                               ten + (size_t)ki * TenStage::COUNT * TenCol<K, R>::ts);
            if (a.rhs) launch_load_boundary<K, R>(m, a, s);
            done = true;
        }
    }
    if (a.vals && !done) hipLaunchKernelGGL((assemble_kernel<K, R>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    if (a.rhs && !done) launch_load_vector<K, R>(m, a, s);
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
    if (parts & ~(uint32_t)(DG_PART_ALL | DG_ASM_MATRIX_CORE)) return DG_ERR_ARG;
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
    a.mL = m->d_gt;
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

// ---------------------------------------------------------------------------
// L2 error of a DG solution (dg_error, section 2.4).
// ---------------------------------------------------------------------------
namespace dg {

__global__ void error_points_kernel(const double* __restrict__ xy, const double* __restrict__ et, int nq, int64_t T,
                                    double* __restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= T * nq) return;
    const int64_t K = idx / nq;
    const int g = (int)(idx - K * nq);
    const double* p = xy + 6 * K;
    const double xi = et[nq + g], eta = et[2 * nq + g];
    out[2 * idx] = p[0] + (p[2] - p[0]) * xi + (p[4] - p[0]) * eta;
    out[2 * idx + 1] = p[1] + (p[3] - p[1]) * xi + (p[5] - p[1]) * eta;
}

// Fixed grid of ERR_BLOCKS workgroups striding over (element, point) pairs:
// the order of every sum is fixed by the launch, so the result is
// deterministic.  part[b] = sum of w_g det_K (u_h - u)^2 over block b's pairs.
__global__ __launch_bounds__(256) void l2_error_kernel(const double* __restrict__ xy, const double* __restrict__ et,
                                                       int nq, int n, int64_t T, const double* __restrict__ x,
                                                       const double* __restrict__ exact, double* __restrict__ part)
{
    __shared__ double sh[4];
    double acc = 0.0;
    const int64_t tot = T * nq;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < tot; idx += (int64_t)ERR_BLOCKS * 256) {
        const int64_t K = idx / nq;
        const int g = (int)(idx - K * nq);
        const double* p = xy + 6 * K;
        const double det = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
        const double* phi = et + 3 * nq + (int64_t)g * n;
        double uh = 0.0;
        for (int m = 0; m < n; ++m) uh += x[K * n + m] * phi[m];
        const double d = uh - exact[idx];
        acc += et[g] * det * d * d;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void sum_parts_kernel(double* part)
{
    __shared__ double sh[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < ERR_BLOCKS; i += 256) acc += part[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[ERR_BLOCKS] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace dg

extern "C" int32_t dg_mesh_error_points(const dg_mesh* m, double* dev_xy, void* stream)
{
    if (!m || !dev_xy) return DG_ERR_ARG;
    const int64_t tot = m->T * m->nqr;
    if (tot > 0)
        hipLaunchKernelGGL(dg::error_points_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                           (hipStream_t)stream, m->d_xy, m->d_etab, m->nqr, m->T, dev_xy);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_l2_error(const dg_mesh* m, const double* dev_x, const double* dev_exact, double* l2,
                               double* h_max, void* stream)
{
    if (!m || !dev_x || !dev_exact) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(dg::l2_error_kernel, dim3(dg::ERR_BLOCKS), dim3(256), 0, s, m->d_xy, m->d_etab, m->nqr, m->n,
                       m->T, dev_x, dev_exact, m->d_epart);
    hipLaunchKernelGGL(dg::sum_parts_kernel, dim3(1), dim3(256), 0, s, m->d_epart);
    double ssq = 0.0;
    DG_HIP_CHECK(hipGetLastError());
    DG_HIP_CHECK(hipMemcpyAsync(&ssq, m->d_epart + dg::ERR_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    if (!std::isfinite(ssq)) return DG_ERR_NONFINITE;
    if (l2) *l2 = std::sqrt(ssq);
    if (h_max) *h_max = m->hmax;
    return DG_OK;
}
