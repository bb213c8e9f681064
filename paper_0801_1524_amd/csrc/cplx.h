// Device helpers: complex arithmetic on HIP vector types and reads of
// read-only tables through the constant address space.
#pragma once

#include <hip/hip_runtime.h>

namespace bfsft {

template <typename T> struct CV;
template <> struct CV<double> { using t = double2; };
template <> struct CV<float> { using t = float2; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += a * b
template <typename V> __device__ __forceinline__ void cfma(V &acc, const V a, const V b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

// acc += r * b for a real r
template <typename R, typename V> __device__ __forceinline__ void rfma(V &acc, const R r, const V b)
{
    acc.x = fma(r, b.x, acc.x);
    acc.y = fma(r, b.y, acc.y);
}

template <typename V> __device__ __forceinline__ V czero()
{
    V r;
    r.x = 0;
    r.y = 0;
    return r;
}

template <typename V> __device__ __forceinline__ V cadd(V a, V b)
{
    a.x += b.x;
    a.y += b.y;
    return a;
}

template <typename D, typename Sv> __device__ __forceinline__ D cvt(const Sv s)
{
    D r;
    r.x = s.x;
    r.y = s.y;
    return r;
}

// Read-only operator tables are addressed through the constant address
// space: wave-uniform loads from it become scalar loads, so table entries
// arrive in SGPRs and feed the FMAs directly.
template <typename T> using cptr = const __attribute__((address_space(4))) T *;

// complex entry i of a constant-address-space table of interleaved scalars
template <typename Cv, typename T> __device__ __forceinline__ Cv ldc(cptr<T> p, int i)
{
    Cv r;
    r.x = p[2 * i];
    r.y = p[2 * i + 1];
    return r;
}

}  // namespace bfsft
