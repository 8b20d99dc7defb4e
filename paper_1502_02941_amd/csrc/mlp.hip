// Small multilayer perceptron for the learned initial guess (gfx950).
//
// Layers l = 1..L: Z_l = H_{l-1} W_l^T + b_l, H_l = silu(Z_l) (no activation
// on the last layer).  Weights are kept in FP32 (master copy, Adam moments)
// and rounded to BF16 for every product; products accumulate in FP32 on the
// MFMA units (v_mfma_f32_16x16x32_bf16: one wavefront computes a 32x32 output
// tile as 2x2 blocks of 16x16).  Activations that feed a product are stored
// in BF16, pre-activations in FP32.  Backward: dZ_L = dY; dW_l = dZ_l^T
// H_{l-1}; db_l = sum over the batch of dZ_l; dH_{l-1} = dZ_l W_l;
// dZ_{l-1} = dH_{l-1} * silu'(Z_{l-1}); the dZ operands of the products are
// rounded to BF16, the bias gradients are summed from FP32 dZ.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "dg_internal.h"

namespace dg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet)
__host__ __device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ __forceinline__ float bf2f(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_d(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C(m,n) = sum_k A(m,k) B(k,n): A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
// (BF16 bits).  Epilogue: + bias[n]; Z (FP32, may be null) = result;
// H (BF16, may be null) = act ? silu(result) : result.
struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int64_t sam, sak, sbk, sbn;
    int M, N, K;
    const float* bias;
    float* Z;
    uint16_t* H;
    int ldc;
    int act;
};

// How an operand tile is read from global memory: its 8-element runs along k
// are contiguous (KRUN), or along the tile's row/column index (XRUN: m for A,
// n for B), each run a 16-byte load; otherwise element by element (SCALAR).
enum { SCALAR = 0, KRUN = 1, XRUN = 2 };
constexpr int GT = 32, GLD = GT + 8;  // tile edge; LDS row stride in BF16 (80 bytes: rows start on 16-byte words)

// One operand tile T[x][k] (x = m or n, 32 x 32, k contiguous in LDS) of
// X(x, k) = P[x * sx + k * sk], zero outside x < X, k < K.  64 lanes, two
// 16-byte runs each.
template <int MODE>
__device__ __forceinline__ void stage_tile(uint16_t (*T)[GLD], const uint16_t* __restrict__ P, int64_t sx, int64_t sk,
                                           int x0, int X, int k0, int K, int lane)
{
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int c = lane + 64 * r;
        if (MODE == KRUN) {  // run c: row x0 + c / 4, k = k0 + 8 (c % 4) .. + 7
            const int x = x0 + (c >> 2), kk = k0 + 8 * (c & 3);
            uint4 v = {0u, 0u, 0u, 0u};
            if (x < X && kk + 8 <= K) {
                v = *reinterpret_cast<const uint4*>(P + (int64_t)x * sx + kk);
            } else if (x < X) {
                uint16_t e[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) e[q] = kk + q < K ? P[(int64_t)x * sx + kk + q] : 0;
                memcpy(&v, e, 16);
            }
            *reinterpret_cast<uint4*>(&T[c >> 2][8 * (c & 3)]) = v;
        } else if (MODE == XRUN) {  // run c: k = k0 + c / 4, x = x0 + 8 (c % 4) .. + 7, transposed into T
            const int kk = k0 + (c >> 2), x = x0 + 8 * (c & 3);
            uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (kk < K && x + 8 <= X) {
                const uint4 v = *reinterpret_cast<const uint4*>(P + (int64_t)kk * sk + x);
                memcpy(e, &v, 16);
            } else if (kk < K) {
#pragma unroll
                for (int q = 0; q < 8; ++q) e[q] = x + q < X ? P[(int64_t)kk * sk + x + q] : 0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) T[8 * (c & 3) + q][c >> 2] = e[q];
        } else {  // element by element: x = c / 4, k = 8 (c % 4) .. + 7
            const int x = x0 + (c >> 2), kk = k0 + 8 * (c & 3);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                T[c >> 2][8 * (c & 3) + q] = (x < X && kk + q < K) ? P[(int64_t)x * sx + (int64_t)(kk + q) * sk] : 0;
        }
    }
}

// One wavefront per 32 x 32 output tile (2 x 2 MFMA blocks of 16 x 16); per
// k-step of 32 both operand tiles go through LDS and each lane reads its
// operand (row or column lane % 16, k = 8 (lane / 16) .. + 7) as one 16-byte word.
template <int AM, int BM>
__global__ __launch_bounds__(64) void gemm_bf16_kernel(const GemmArgs g)
{
    __shared__ __align__(16) uint16_t As[GT][GLD];
    __shared__ __align__(16) uint16_t Bs[GT][GLD];
    const int lane = threadIdx.x;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    f32x4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += GT) {
        stage_tile<AM>(As, g.A, g.sam, g.sak, m0, g.M, k0, g.K, lane);
        stage_tile<BM>(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, g.K, lane);
        __syncthreads();
        bf16x8_t av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            av[t] = *reinterpret_cast<const bf16x8_t*>(&As[16 * t + r16][kq]);
            bv[t] = *reinterpret_cast<const bf16x8_t*>(&Bs[16 * t + r16][kq]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        __syncthreads();  // the next k-step overwrites the tiles
    }
    // result lane layout: column = lane%16, rows 4*(lane/16)..+3
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + 16 * a + 4 * (lane >> 4) + i, n = n0 + 16 * b + r16;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[a][b][i] + (g.bias ? g.bias[n] : 0.f);
                if (g.Z) g.Z[(int64_t)m * g.ldc + n] = v;
                if (g.H) g.H[(int64_t)m * g.ldc + n] = f2bf(g.act ? silu(v) : v);
            }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// dZ = dH * silu'(Z) (FP32) and its BF16 copy
__global__ void act_back_kernel(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                                uint16_t* __restrict__ dZb, int64_t n, int act)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = act ? dH[i] * silu_d(Z[i]) : dH[i];
    dZ[i] = v;
    dZb[i] = f2bf(v);
}

// db[n] = sum_b dZ[b][n]
__global__ void bias_grad_kernel(const float* __restrict__ dZ, int B, int N, float* __restrict__ db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + n];
    db[n] = s;
}

// dY = 2 (Y - T) / (B * N), loss partials (sum of squares / (B * N))
__global__ void mse_kernel(const float* __restrict__ Y, const float* __restrict__ T, int64_t n, float scale,
                           float* __restrict__ dY, float* __restrict__ part)
{
    __shared__ float sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const float d = Y[i] - T[i];
        dY[i] = 2.f * d * scale;
        l = d * d * scale;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void sum_kernel(const float* __restrict__ part, int n, float* out)
{
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 64) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (threadIdx.x == 0) *out = s;
}

// Adam on the flat FP32 parameters, BF16 copy of the weights refreshed
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m1,
                            float* __restrict__ m2, uint16_t* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float a = b1 * m1[i] + (1.f - b1) * g;
    const float v = b2 * m2[i] + (1.f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    const float q = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[i] = q;
    pb[i] = f2bf(q);
}

// P0 -> P1 initial guess on a mesh from values on an nc x nc grid of cells of
// the unit square.  mode 0: each element takes its cell's value (constant
// mode only: c0 = value / phi0, phi0 the constant basis function: sqrt 2 for
// the orthonormal basis, 1 for the monomials); mode 1: the continuous piecewise bilinear
// interpolant of the cell-centre values (zero on the boundary) at the three
// vertices, then the element's P1 coefficients c_m = sum_v P[m][v] u_v.
__global__ void prolong_kernel(const double* __restrict__ xy, int64_t T, int nloc, const float* __restrict__ coarse,
                               int B, int nc, int mode, const double* __restrict__ P, double phi0,
                               double* __restrict__ x, int64_t ldx)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * T) return;
    const int64_t bi = idx / T, el = idx - bi * T;
    const float* cv = coarse + bi * (int64_t)nc * nc;
    const double* p = xy + 6 * el;
    double* out = x + bi * ldx + el * nloc;
    for (int m = 0; m < nloc; ++m) out[m] = 0.0;
    if (mode == 0) {
        const double cx = (p[0] + p[2] + p[4]) / 3.0, cy = (p[1] + p[3] + p[5]) / 3.0;
        const int i = min(nc - 1, max(0, (int)floor(cx * nc))), j = min(nc - 1, max(0, (int)floor(cy * nc)));
        out[0] = (double)cv[j * nc + i] / phi0;
        return;
    }
    double u[3];
    for (int v = 0; v < 3; ++v) {
        // node coordinates of the extended grid: 0, cell centres, 1 (value 0 at 0 and 1)
        const double sx = p[2 * v] * nc - 0.5, sy = p[2 * v + 1] * nc - 0.5;
        const int i0 = (int)floor(sx), j0 = (int)floor(sy);
        const double tx = sx - i0, ty = sy - j0;
        auto val = [&](int i, int j) -> double {
            return (i < 0 || j < 0 || i >= nc || j >= nc) ? 0.0 : (double)cv[j * nc + i];
        };
        // boundary segments [0, 0.5/nc] and [1 - 0.5/nc, 1]: linear to the zero boundary value
        double wx0 = 1.0 - tx, wx1 = tx, wy0 = 1.0 - ty, wy1 = ty;
        if (i0 < 0) { wx1 = p[2 * v] * nc / 0.5; wx0 = 0.0; }
        if (i0 >= nc - 1) { wx0 = (1.0 - p[2 * v]) * nc / 0.5; wx1 = 0.0; }
        if (j0 < 0) { wy1 = p[2 * v + 1] * nc / 0.5; wy0 = 0.0; }
        if (j0 >= nc - 1) { wy0 = (1.0 - p[2 * v + 1]) * nc / 0.5; wy1 = 0.0; }
        u[v] = wx0 * wy0 * val(i0, j0) + wx1 * wy0 * val(i0 + 1, j0) + wx0 * wy1 * val(i0, j0 + 1) +
               wx1 * wy1 * val(i0 + 1, j0 + 1);
    }
    for (int m = 0; m < 3 && m < nloc; ++m) out[m] = P[m * 3 + 0] * u[0] + P[m * 3 + 1] * u[1] + P[m * 3 + 2] * u[2];
}

}  // namespace dg

using namespace dg;

struct dg_mlp {
    int L = 0;
    std::vector<int> w;  // widths [L+1]
    int max_batch = 0;
    int64_t nparam = 0;
    std::vector<int64_t> woff, boff;  // offsets of W_l, b_l in the flat vector
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    uint16_t* pb = nullptr;            // BF16 copy of all parameters (weights used)
    uint16_t* x16 = nullptr;           // input, BF16 [B][w0]
    std::vector<float*> Z;             // pre-activations [B][w_l], l = 1..L
    std::vector<uint16_t*> H;          // BF16 activations [B][w_l], l = 1..L-1
    float *dZ = nullptr, *dH = nullptr; // scratch [B][max w]
    uint16_t* dZb = nullptr;
    float* part = nullptr;
    int last_B = 0;
};

static void mlp_free(dg_mlp* m)
{
    hipFree(m->p); hipFree(m->g); hipFree(m->m1); hipFree(m->m2); hipFree(m->pb); hipFree(m->x16);
    for (auto z : m->Z) hipFree(z);
    for (auto h : m->H) hipFree(h);
    hipFree(m->dZ); hipFree(m->dH); hipFree(m->dZb); hipFree(m->part);
}

extern "C" int32_t dg_mlp_create(const int32_t* widths, int32_t n_widths, int32_t max_batch, const float* init_params,
                                 dg_mlp** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (!widths || n_widths < 2 || n_widths > 16 || max_batch <= 0 || !init_params) return DG_ERR_ARG;
    dg_mlp* m = new (std::nothrow) dg_mlp();
    if (!m) return DG_ERR_OOM;
    m->L = n_widths - 1;
    m->w.assign(widths, widths + n_widths);
    m->max_batch = max_batch;
    int maxw = 0;
    for (int i = 0; i < n_widths; ++i) {
        if (widths[i] <= 0 || widths[i] > 65536) { delete m; return DG_ERR_ARG; }
        maxw = std::max(maxw, widths[i]);
    }
    for (int l = 0; l < m->L; ++l) {
        m->woff.push_back(m->nparam);
        m->nparam += (int64_t)m->w[l + 1] * m->w[l];
        m->boff.push_back(m->nparam);
        m->nparam += m->w[l + 1];
    }
    bool ok = true;
    auto al = [&](void** p, size_t b) { if (ok && hipMalloc(p, std::max<size_t>(b, 16)) != hipSuccess) { *p = nullptr; ok = false; } };
    al((void**)&m->p, 4 * m->nparam);
    al((void**)&m->g, 4 * m->nparam);
    al((void**)&m->m1, 4 * m->nparam);
    al((void**)&m->m2, 4 * m->nparam);
    al((void**)&m->pb, 2 * m->nparam);
    al((void**)&m->x16, 2 * (size_t)max_batch * m->w[0]);
    m->Z.assign(m->L, nullptr);
    m->H.assign(m->L, nullptr);
    for (int l = 0; l < m->L; ++l) {
        al((void**)&m->Z[l], 4 * (size_t)max_batch * m->w[l + 1]);
        al((void**)&m->H[l], 2 * (size_t)max_batch * m->w[l + 1]);
    }
    al((void**)&m->dZ, 4 * (size_t)max_batch * maxw);
    al((void**)&m->dH, 4 * (size_t)max_batch * maxw);
    al((void**)&m->dZb, 2 * (size_t)max_batch * maxw);
    al((void**)&m->part, 4 * (size_t)((max_batch * (int64_t)maxw + 255) / 256 + 1));
    if (!ok) { mlp_free(m); delete m; return DG_ERR_OOM; }
    std::vector<uint16_t> hb(m->nparam);
    for (int64_t i = 0; i < m->nparam; ++i) {
        if (!std::isfinite(init_params[i])) { mlp_free(m); delete m; return DG_ERR_NONFINITE; }
        hb[i] = f2bf(init_params[i]);
    }
    if (hipMemcpy(m->p, init_params, 4 * m->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->pb, hb.data(), 2 * m->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->m1, 0, 4 * m->nparam) != hipSuccess || hipMemset(m->m2, 0, 4 * m->nparam) != hipSuccess ||
        hipMemset(m->g, 0, 4 * m->nparam) != hipSuccess) {
        mlp_free(m); delete m; return DG_ERR_HIP;
    }
    *out = m;
    return DG_OK;
}

extern "C" int64_t dg_mlp_num_params(const dg_mlp* m) { return m ? m->nparam : -1; }

extern "C" void dg_mlp_destroy(dg_mlp* m)
{
    if (!m) return;
    mlp_free(m);
    delete m;
}

// operand read mode: 16-byte runs need a 16-byte aligned base and a run
// stride that keeps every run on a 16-byte word
static int run_mode(const uint16_t* P, int64_t sx, int64_t sk)
{
    if (reinterpret_cast<uintptr_t>(P) % 16 != 0) return SCALAR;
    if (sk == 1 && sx % 8 == 0) return KRUN;
    if (sx == 1 && sk % 8 == 0) return XRUN;
    return SCALAR;
}

template <int AM>
static void launch_gemm_b(int bm, dim3 grid, hipStream_t s, const GemmArgs& g)
{
    if (bm == KRUN) hipLaunchKernelGGL((gemm_bf16_kernel<AM, KRUN>), grid, dim3(64), 0, s, g);
    else if (bm == XRUN) hipLaunchKernelGGL((gemm_bf16_kernel<AM, XRUN>), grid, dim3(64), 0, s, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<AM, SCALAR>), grid, dim3(64), 0, s, g);
}

static void gemm(hipStream_t s, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                 int64_t sbn, int M, int N, int K, const float* bias, float* Z, uint16_t* H, int ldc, int act)
{
    GemmArgs g{A, B, sam, sak, sbk, sbn, M, N, K, bias, Z, H, ldc, act};
    const dim3 grid((M + GT - 1) / GT, (N + GT - 1) / GT);
    const int am = run_mode(A, sam, sak), bm = run_mode(B, sbn, sbk);
    if (am == KRUN) launch_gemm_b<KRUN>(bm, grid, s, g);
    else if (am == XRUN) launch_gemm_b<XRUN>(bm, grid, s, g);
    else launch_gemm_b<SCALAR>(bm, grid, s, g);
}

extern "C" int32_t dg_mlp_forward(dg_mlp* m, const float* dev_x, int32_t B, float* dev_y, void* stream)
{
    if (!m || !dev_x || B <= 0 || B > m->max_batch) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nx = (int64_t)B * m->w[0];
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, dev_x, m->x16, nx);
    const uint16_t* in = m->x16;
    for (int l = 0; l < m->L; ++l) {
        const int K = m->w[l], N = m->w[l + 1];
        const bool last = l == m->L - 1;
        gemm(s, in, K, 1, m->pb + m->woff[l], 1, K, B, N, K, m->p + m->boff[l], m->Z[l], last ? nullptr : m->H[l], N,
             last ? 0 : 1);
        in = m->H[l];
    }
    const int No = m->w[m->L];
    if (dev_y) DG_HIP_CHECK(hipMemcpyAsync(dev_y, m->Z[m->L - 1], 4 * (size_t)B * No, hipMemcpyDeviceToDevice, s));
    m->last_B = B;
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_mlp_loss_mse(dg_mlp* m, const float* dev_target, int32_t B, float* dev_dy, float* dev_loss,
                                   void* stream)
{
    if (!m || !dev_target || !dev_dy || !dev_loss || B != m->last_B) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)B * m->w[m->L];
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, m->Z[m->L - 1], dev_target, n, 1.0f / (float)n, dev_dy,
                       m->part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s, m->part, nb, dev_loss);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_mlp_backward(dg_mlp* m, const float* dev_dy, int32_t B, void* stream)
{
    if (!m || !dev_dy || B != m->last_B) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const float* dcur = dev_dy;  // gradient w.r.t. Z_l (FP32)
    for (int l = m->L - 1; l >= 0; --l) {
        const int K = m->w[l], N = m->w[l + 1];
        const int64_t n = (int64_t)B * N;
        // dZ_l: for the last layer dY itself; otherwise dH_l * silu'(Z_l)
        hipLaunchKernelGGL(act_back_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dcur, m->Z[l], m->dZ,
                           m->dZb, n, l == m->L - 1 ? 0 : 1);
        hipLaunchKernelGGL(bias_grad_kernel, dim3((N + 255) / 256), dim3(256), 0, s, (const float*)m->dZ, B, N,
                           m->g + m->boff[l]);
        // dW_l (N x K) = dZ_l^T (N x B) H_{l-1} (B x K)
        const uint16_t* Hin = l == 0 ? m->x16 : m->H[l - 1];
        gemm(s, m->dZb, 1, N, Hin, K, 1, N, K, B, nullptr, m->g + m->woff[l], nullptr, K, 0);
        if (l > 0) {
            // dH_{l-1} (B x K) = dZ_l (B x N) W_l (N x K)
            gemm(s, m->dZb, N, 1, m->pb + m->woff[l], K, 1, B, K, N, nullptr, m->dH, nullptr, K, 0);
            dcur = m->dH;
        }
    }
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_mlp_adam_step(dg_mlp* m, float lr, float beta1, float beta2, float eps, int32_t t, void* stream)
{
    if (!m || t < 1 || !(lr >= 0)) return DG_ERR_ARG;
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((m->nparam + 255) / 256)), dim3(256), 0, (hipStream_t)stream, m->p,
                       (const float*)m->g, m->m1, m->m2, m->pb, m->nparam, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}

extern "C" int32_t dg_mlp_params(dg_mlp* m, float* dev_params, float* dev_grads, void* stream)
{
    if (!m) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (dev_params) DG_HIP_CHECK(hipMemcpyAsync(dev_params, m->p, 4 * m->nparam, hipMemcpyDeviceToDevice, s));
    if (dev_grads) DG_HIP_CHECK(hipMemcpyAsync(dev_grads, m->g, 4 * m->nparam, hipMemcpyDeviceToDevice, s));
    return DG_OK;
}

extern "C" int32_t dg_warmstart_prolong(const dg_mesh* mesh, const float* dev_coarse, int32_t B, int32_t nc,
                                        int32_t mode, double* dev_x, int64_t ldx, void* stream)
{
    if (!mesh || !dev_coarse || !dev_x || B <= 0 || nc <= 0 || (mode != 0 && mode != 1)) return DG_ERR_ARG;
    if (mesh->k < 1 && mode == 1) return DG_ERR_DEGREE;
    if (ldx < mesh->T * mesh->n) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int64_t tot = (int64_t)B * mesh->T;
    hipLaunchKernelGGL(prolong_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, mesh->d_xy, mesh->T,
                       mesh->n, dev_coarse, B, nc, mode, (const double*)mesh->d_p1map, mesh->phi0, dev_x, ldx);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DG_OK : DG_ERR_HIP;
}
