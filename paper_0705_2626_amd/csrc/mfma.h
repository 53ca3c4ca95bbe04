// 16x16x4 MFMA helpers for gfx950 (wave64).
//
// D (16x16) += A (16x4) B (4x16).  Operands: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16].  Accumulator register r of lane l holds
// D[row(l, r)][l % 16] with
//   f32_16x16x4f32: row = 4 * (l / 16) + r
//   f64_16x16x4f64: row = l / 16 + 4 * r
// (the two layouts differ; both were checked on the device).
#pragma once

#include <hip/hip_runtime.h>

namespace lobpcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<float> {
    typedef floatx4 acc;
    static __device__ __forceinline__ floatx4 mma(float a, float b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <>
struct Mfma<double> {
    typedef doublex4 acc;
    static __device__ __forceinline__ doublex4 mma(double a, double b, doublex4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T>
__device__ __forceinline__ typename Mfma<T>::acc acc_zero()
{
    typename Mfma<T>::acc z;
#pragma unroll
    for (int r = 0; r < 4; r++) z[r] = T(0);
    return z;
}

}  // namespace lobpcg
