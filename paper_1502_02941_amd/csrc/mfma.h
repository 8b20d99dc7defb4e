// Matrix-core (MFMA) 16 x 16 x 4 products in FP64 and FP32 as used by the
// assembly and the block Gram-Schmidt kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace dg {

// Both take A[i][k] from lane i + 16 k and B[k][j] from lane j + 16 k, and
// leave D[i][j] in lane j + 16 g, register v: the FP64 product with rows
// i = g + 4 v, the FP32 one with rows i = 4 g + v (measured on gfx950).
template <typename R>
struct MfmaOp;
template <>
struct MfmaOp<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V mac(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
    static __device__ __forceinline__ void store(double x, __amdgpu_buffer_rsrc_t rs, uint32_t off)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(MfU2, x), rs, (int)off, 0, 0);
    }
    typedef unsigned int MfU2 __attribute__((ext_vector_type(2)));
};
template <>
struct MfmaOp<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V mac(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
    static __device__ __forceinline__ void store(float x, __amdgpu_buffer_rsrc_t rs, uint32_t off)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), rs, (int)off, 0, 0);
    }
};

}  // namespace dg
