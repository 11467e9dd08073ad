// surface_common.hpp -- the per-vertex surface arithmetic and store helpers
// shared by the single-sweep and batched surface kernels.
#pragma once

#include "kernels.hpp"

namespace sweep {

template <bool NT, class T>
__device__ __forceinline__ void store_one(T* p, T v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <class T> __device__ __forceinline__ T inv_norm(T n2);
template <> __device__ __forceinline__ float inv_norm<float>(float n2)
{
    return (n2 > 0.0f && n2 < INFINITY) ? rsqrtf(n2) : 0.0f;
}
template <> __device__ __forceinline__ double inv_norm<double>(double n2)
{
    return (n2 > 0.0 && n2 < INFINITY) ? 1.0 / sqrt(n2) : 0.0;
}

// One vertex from a row record (x r s t L a b) and a profile record (S S').
template <class T>
__device__ __forceinline__ void vertex(const T* row, T Sx, T Sy, T Sz, T Dx, T Dy, T Dz, T* X, T* Nn)
{
    const T x0 = row[0], x1 = row[1], x2 = row[2];
    const T r0 = row[3], r1 = row[4], r2 = row[5];
    const T s0 = row[6], s1 = row[7], s2 = row[8];
    const T t0 = row[9], t1 = row[10], t2 = row[11];
    const T L = row[12], a = row[13], b = row[14];
    X[0] = x0 + Sx * r0 + Sy * s0 + Sz * t0;
    X[1] = x1 + Sx * r1 + Sy * s1 + Sz * t1;
    X[2] = x2 + Sx * r2 + Sy * s2 + Sz * t2;
    const T ux = Sz * a, uy = Sz * b, uz = L - Sx * a - Sy * b;
    T nx = Dy * uz - Dz * uy;
    T ny = Dz * ux - Dx * uz;
    T nz = Dx * uy - Dy * ux;
    const T inv = inv_norm<T>(nx * nx + ny * ny + nz * nz);
    nx *= inv; ny *= inv; nz *= inv;
    Nn[0] = nx * r0 + ny * s0 + nz * t0;
    Nn[1] = nx * r1 + ny * s1 + nz * t1;
    Nn[2] = nx * r2 + ny * s2 + nz * t2;
}

template <bool NT, class T>
__device__ __forceinline__ void store6(T* __restrict__ pos, T* __restrict__ nrm, size_t N, size_t v,
                                       const T* X, const T* Nn, bool wn)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) store_one<NT>(pos + c * N + v, X[c]);
    if (wn) {
#pragma unroll
        for (int c = 0; c < 3; ++c) store_one<NT>(nrm + c * N + v, Nn[c]);
    }
}

// floor(v / d) for 0 <= v < 2^31 by one 64-bit multiply and shift.
struct FastDiv {
    unsigned long long m;
    int shift;
    int d;
};

__device__ __forceinline__ int fdiv(unsigned v, const FastDiv& f)
{
    return (int)(((unsigned long long)v * f.m) >> f.shift);
}

// Rows touched by a block of 256*K consecutive vertices: at most
// 256*K/n_v + 2.  Up to kMaxLdsRows are staged in LDS; a block that touches
// more (tiny n_v with large K) reads its rows from global memory instead.
constexpr int kMaxLdsRows = 144;

}  // namespace sweep
