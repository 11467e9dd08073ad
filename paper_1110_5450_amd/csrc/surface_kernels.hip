// surface_kernels.hip -- the surface write (the hot loop): for every vertex
//   X = x_i + S_x r_i + S_y s_i + S_z t_i
//   N = R_i normalize(S'_j x (S_z a_i, S_z b_i, |C'_i| - S_x a_i - S_y b_i))
// where the cross product is taken in frame coordinates (X_v = R S',
// X_u = R (S_z a, S_z b, alpha) with t' = a r + b s), and written as six
// SoA planes.  The work is bound by HBM write bandwidth (24 B per vertex in
// FP32, 48 B in FP64); loads are a 64-byte row record per u-row and a
// 32-byte profile record per v-sample, both cache resident.
//
// kind 0 (column-stationary): each thread owns 4 consecutive columns, keeps
//   their profile records in registers and walks a group of rows; the row
//   record is uniform across the block (scalar loads) and every plane store
//   is a 16-byte vector store, 1 KiB contiguous per wave.  Needs n_v % 4 == 0
//   and 16-byte aligned outputs.
// kind 1 (linear): each thread takes vertices v = tile*TV + tid + 256*k of
//   the flattened grid; row and profile records are per-lane loads and every
//   plane store is a 4-byte store, 256 B contiguous per wave.  Any shape.
#include "kernels.hpp"

namespace sweep {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <class T> struct Vec4;
template <> struct Vec4<float> { typedef f4v type; };
template <> struct Vec4<double> { typedef d4v type; };

template <bool NT, class V>
__device__ __forceinline__ void store_vec(V* p, V v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
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

template <class T, bool NRM, bool NT>
__global__ __launch_bounds__(kBlock) void k_surface_cols(const T* __restrict__ rows, const T* __restrict__ prof,
                                                         int n_u, int n_v, int rows_per_block, int n_col_tiles,
                                                         T* __restrict__ pos, T* __restrict__ nrm)
{
    typedef typename Vec4<T>::type V;
    const int ct = blockIdx.x % n_col_tiles;
    const int rg = blockIdx.x / n_col_tiles;
    const int j0 = (ct * kBlock + threadIdx.x) * 4;
    if (j0 >= n_v) return;
    T Sx[4], Sy[4], Sz[4], Dx[4], Dy[4], Dz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T* q = prof + 8 * (size_t)(j0 + k);
        Sx[k] = q[0]; Sy[k] = q[1]; Sz[k] = q[2];
        Dx[k] = q[3]; Dy[k] = q[4]; Dz[k] = q[5];
    }
    const int i0 = rg * rows_per_block;
    const int i1 = min(n_u, i0 + rows_per_block);
    const size_t N = (size_t)n_u * (size_t)n_v;
    for (int i = i0; i < i1; ++i) {
        const T* row = rows + 16 * (size_t)i;
        T X[4][3], Nn[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) vertex<T>(row, Sx[k], Sy[k], Sz[k], Dx[k], Dy[k], Dz[k], X[k], Nn[k]);
        const size_t off = (size_t)i * (size_t)n_v + (size_t)j0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            V v = {X[0][c], X[1][c], X[2][c], X[3][c]};
            store_vec<NT>((V*)(pos + c * N + off), v);
        }
        if (NRM) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                V v = {Nn[0][c], Nn[1][c], Nn[2][c], Nn[3][c]};
                store_vec<NT>((V*)(nrm + c * N + off), v);
            }
        }
    }
}

// floor(v / d) for 0 <= v < 2^31 by one 64-bit multiply and shift.
struct FastDiv {
    unsigned long long m;
    int shift;
    int d;
};

static FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1LL << l) < d) ++l;
    const int sh = 31 + l;
    // m = ceil(2^sh / d)
    const unsigned __int128 num = (unsigned __int128)1 << sh;
    const unsigned long long m = (unsigned long long)((num + (unsigned)d - 1) / (unsigned)d);
    return FastDiv{m, sh, d};
}

__device__ __forceinline__ int fdiv(unsigned v, const FastDiv& f)
{
    return (int)(((unsigned long long)v * f.m) >> f.shift);
}

template <class T, bool NRM, bool NT>
__global__ __launch_bounds__(kBlock) void k_surface_linear(const T* __restrict__ rows, const T* __restrict__ prof,
                                                           int n_u, int n_v, FastDiv dv, int tile_vertices,
                                                           int n_tiles, T* __restrict__ pos, T* __restrict__ nrm)
{
    const long long N = (long long)n_u * (long long)n_v;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const long long base = (long long)tile * tile_vertices;
        const long long end = min(N, base + tile_vertices);
        for (long long v = base + threadIdx.x; v < end; v += kBlock) {
            const int i = fdiv((unsigned)v, dv);
            const int j = (int)v - i * n_v;
            const T* q = prof + 8 * (size_t)j;
            T X[3], Nn[3];
            vertex<T>(rows + 16 * (size_t)i, q[0], q[1], q[2], q[3], q[4], q[5], X, Nn);
#pragma unroll
            for (int c = 0; c < 3; ++c) store_one<NT>(pos + c * N + v, X[c]);
            if (NRM) {
#pragma unroll
                for (int c = 0; c < 3; ++c) store_one<NT>(nrm + c * N + v, Nn[c]);
            }
        }
    }
}

bool surface_cols_supported(int n_v, const void* pos, const void* nrm, size_t elem)
{
    (void)elem;
    if (n_v % 4 != 0) return false;
    if (((uintptr_t)pos) % 16 != 0) return false;
    if (nrm && ((uintptr_t)nrm) % 16 != 0) return false;
    return true;
}

template <class T, bool NRM, bool NT>
static void launch_surface_t(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                             const SurfaceConfig& cfg, hipStream_t st)
{
    if (cfg.kind == 0) {
        const int n_col_tiles = (n_v + 4 * kBlock - 1) / (4 * kBlock);
        const int rpb = cfg.rows_per_block > 0 ? cfg.rows_per_block : 16;
        const int n_row_groups = (n_u + rpb - 1) / rpb;
        hipLaunchKernelGGL((k_surface_cols<T, NRM, NT>), dim3(n_col_tiles * n_row_groups), dim3(kBlock), 0, st,
                           rows, prof, n_u, n_v, rpb, n_col_tiles, pos, nrm);
    } else {
        const long long N = (long long)n_u * n_v;
        const int tv = cfg.tile_vertices > 0 ? cfg.tile_vertices : 4096;
        const int n_tiles = (int)((N + tv - 1) / tv);
        const int grid = cfg.grid > 0 ? min(cfg.grid, n_tiles) : n_tiles;
        hipLaunchKernelGGL((k_surface_linear<T, NRM, NT>), dim3(grid), dim3(kBlock), 0, st, rows, prof, n_u, n_v,
                           make_fastdiv(n_v), tv, n_tiles, pos, nrm);
    }
}

template <class T>
hipError_t launch_surface(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                          const SurfaceConfig& cfg, hipStream_t st)
{
    const bool wn = nrm != nullptr;
    if (cfg.nontemporal) {
        if (wn) launch_surface_t<T, true, true>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
        else launch_surface_t<T, false, true>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    } else {
        if (wn) launch_surface_t<T, true, false>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
        else launch_surface_t<T, false, false>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    }
    return hipGetLastError();
}
template hipError_t launch_surface<float>(const float*, const float*, int, int, float*, float*,
                                          const SurfaceConfig&, hipStream_t);
template hipError_t launch_surface<double>(const double*, const double*, int, int, double*, double*,
                                           const SurfaceConfig&, hipStream_t);

}  // namespace sweep
