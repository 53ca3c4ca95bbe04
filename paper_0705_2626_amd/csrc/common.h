// Shared device helpers for the LOBPCG kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lobpcg {

typedef long long i64;

// V consecutive elements of one grid point's row, moved as one 16/8/4-byte access.
template <typename T, int V>
struct alignas(sizeof(T) * V) vec {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ vec<T, V> vzero()
{
    vec<T, V> r;
#pragma unroll
    for (int i = 0; i < V; i++) r.v[i] = T(0);
    return r;
}

template <typename T, int V>
__device__ __forceinline__ vec<T, V> vload(const T *p)
{
    return *reinterpret_cast<const vec<T, V> *>(p);
}

template <typename T, int V>
__device__ __forceinline__ void vstore(T *p, const vec<T, V> &x)
{
    *reinterpret_cast<vec<T, V> *>(p) = x;
}

// The same store marked non-temporal: streamed results that should not
// displace operands still to be re-read from the caches.
template <typename T, int V>
__device__ __forceinline__ void vstore_nt(T *p, const vec<T, V> &x)
{
    typedef T vt __attribute__((ext_vector_type(V)));
    vt v;
#pragma unroll
    for (int i = 0; i < V; i++) v[i] = x.v[i];
    __builtin_nontemporal_store(v, reinterpret_cast<vt *>(p));
}

// Workgroup -> tile remap so that consecutive tiles run on one XCD.  The
// hardware deals workgroups round-robin over the 8 XCDs (workgroup b lands on
// XCD b % 8); giving each XCD a contiguous range of tiles keeps neighbouring
// tiles (and their shared halo rows) in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb)
{
    const unsigned nx = 8;
    if (nb % nx) return b;
    return (b % nx) * (nb / nx) + b / nx;
}

}  // namespace lobpcg
