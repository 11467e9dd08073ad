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

// One vertex from an extended row record (32 values: x r s t L a b omega
// A A' sigma sigma') and a profile record (S S'): the profile point in the
// frame is p = (A (S_x, S_y), sigma S_z), its u-derivative
// p' = (A' (S_x, S_y), sigma' S_z), and in frame coordinates
//   X_v = (A (S'_x, S'_y), sigma S'_z),
//   X_u = (p'_r + p_t a - omega p_s, p'_s + p_t b + omega p_r,
//          L - p_r a - p_s b + p'_t).
template <class T>
__device__ __forceinline__ void vertex_ext(const T* row, T Sx, T Sy, T Sz, T Dx, T Dy, T Dz, T* X, T* Nn)
{
    const T x0 = row[0], x1 = row[1], x2 = row[2];
    const T r0 = row[3], r1 = row[4], r2 = row[5];
    const T s0 = row[6], s1 = row[7], s2 = row[8];
    const T t0 = row[9], t1 = row[10], t2 = row[11];
    const T L = row[12], a = row[13], b = row[14], om = row[15];
    const T A00 = row[16], A01 = row[17], A10 = row[18], A11 = row[19];
    const T G00 = row[20], G01 = row[21], G10 = row[22], G11 = row[23];
    const T sg = row[24], dsg = row[25];
    const T pr = A00 * Sx + A01 * Sy, ps = A10 * Sx + A11 * Sy, pt = sg * Sz;
    const T dpr = G00 * Sx + G01 * Sy, dps = G10 * Sx + G11 * Sy, dpt = dsg * Sz;
    X[0] = x0 + pr * r0 + ps * s0 + pt * t0;
    X[1] = x1 + pr * r1 + ps * s1 + pt * t1;
    X[2] = x2 + pr * r2 + ps * s2 + pt * t2;
    const T qx = A00 * Dx + A01 * Dy, qy = A10 * Dx + A11 * Dy, qz = sg * Dz;
    const T ux = dpr + pt * a - om * ps, uy = dps + pt * b + om * pr, uz = L - pr * a - ps * b + dpt;
    T nx = qy * uz - qz * uy;
    T ny = qz * ux - qx * uz;
    T nz = qx * uy - qy * ux;
    const T inv = inv_norm<T>(nx * nx + ny * ny + nz * nz);
    nx *= inv; ny *= inv; nz *= inv;
    Nn[0] = nx * r0 + ny * s0 + nz * t0;
    Nn[1] = nx * r1 + ny * s1 + nz * t1;
    Nn[2] = nx * r2 + ny * s2 + nz * t2;
}

// Row record length RL (16 or 32) selects the vertex formula.
template <int RL, class T>
__device__ __forceinline__ void vertex_rl(const T* row, T Sx, T Sy, T Sz, T Dx, T Dy, T Dz, T* X, T* Nn)
{
    if (RL == 16) vertex<T>(row, Sx, Sy, Sz, Dx, Dy, Dz, X, Nn);
    else vertex_ext<T>(row, Sx, Sy, Sz, Dx, Dy, Dz, X, Nn);
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
