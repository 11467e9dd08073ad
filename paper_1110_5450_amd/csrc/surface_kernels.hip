// surface_kernels.hip -- the surface write (the hot loop): for every vertex
//   X = x_i + S_x r_i + S_y s_i + S_z t_i
//   N = R_i normalize(S'_j x (S_z a_i, S_z b_i, |C'_i| - S_x a_i - S_y b_i))
// where the cross product is taken in frame coordinates (X_v = R S',
// X_u = R (S_z a, S_z b, alpha) with t' = a r + b s), and written as six
// SoA planes.  The work is bound by HBM write bandwidth (24 B per vertex in
// FP32, 48 B in FP64); the inputs are a 16-value row record per u-row and an
// 8-value profile record per v-sample, both cache resident.
//
// Measured on MI355X, six interleaved store streams reach ~6.0-6.3 TB/s when
// every block writes about 1 KiB per plane and then retires (many small
// blocks keep the most stores in flight); longer-lived blocks and 16-byte
// stores per lane were not faster.  Both kernels therefore give each lane one
// vertex per row step and store one element per plane, so a wave's store
// covers 256 B (FP32) or 512 B (FP64) contiguous bytes.
//
// kind 0 (column tiles): a block covers 256 consecutive columns of R rows;
//   each lane keeps its column's profile record in registers and the row
//   record is block-uniform (scalar loads).  For n_v >= 256.
// kind 1 (linear): a block covers 256*K consecutive vertices of the flattened
//   grid (lane-contiguous); the rows it touches are staged in LDS and each
//   lane reads its profile record from the (cached) table.  Any shape.
#include "surface_common.hpp"

namespace sweep {

template <class T, bool NRM, bool NT, int RL>
__global__ __launch_bounds__(kBlock) void k_surface_tiles(const T* __restrict__ rows, const T* __restrict__ prof,
                                                          int n_u, int n_v, int R, int n_col_tiles,
                                                          T* __restrict__ pos, T* __restrict__ nrm)
{
    const int ct = blockIdx.x % n_col_tiles;
    const int rg = blockIdx.x / n_col_tiles;
    const int j = ct * kBlock + threadIdx.x;
    if (j >= n_v) return;
    const T* q = prof + 8 * (size_t)j;
    const T Sx = q[0], Sy = q[1], Sz = q[2], Dx = q[3], Dy = q[4], Dz = q[5];
    const int i0 = rg * R;
    const int i1 = min(n_u, i0 + R);
    const size_t N = (size_t)n_u * (size_t)n_v;
    for (int i = i0; i < i1; ++i) {
        T X[3], Nn[3];
        vertex_rl<RL, T>(rows + RL * (size_t)i, Sx, Sy, Sz, Dx, Dy, Dz, X, Nn);
        store6<NT>(pos, nrm, N, (size_t)i * (size_t)n_v + (size_t)j, X, Nn, NRM);
    }
}

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

void fastdiv_constants(int d, unsigned long long* m, int* shift)
{
    const FastDiv f = make_fastdiv(d);
    *m = f.m;
    *shift = f.shift;
}

template <class T, bool NRM, bool NT, int K, int RL>
__global__ __launch_bounds__(kBlock) void k_surface_linear(const T* __restrict__ rows, const T* __restrict__ prof,
                                                           int n_u, int n_v, FastDiv dv,
                                                           T* __restrict__ pos, T* __restrict__ nrm)
{
    __shared__ T lrow[kMaxLdsRows * RL];
    const long long N = (long long)n_u * (long long)n_v;
    const long long v0 = (long long)blockIdx.x * (kBlock * K);
    const long long vlast = min(N, v0 + kBlock * K) - 1;
    const int ilo = fdiv((unsigned)v0, dv);
    const int nrow = fdiv((unsigned)vlast, dv) - ilo + 1;
    const bool staged = nrow <= kMaxLdsRows;
    if (staged)
        for (int e = threadIdx.x; e < nrow * RL; e += kBlock) lrow[e] = rows[RL * (size_t)ilo + e];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long v = v0 + threadIdx.x + k * kBlock;
        if (v < N) {
            const int i = fdiv((unsigned)v, dv);
            const int j = (int)v - i * n_v;
            const T* q = prof + 8 * (size_t)j;
            T X[3], Nn[3];
            const T* row = staged ? lrow + RL * (i - ilo) : rows + RL * (size_t)i;
            vertex_rl<RL, T>(row, q[0], q[1], q[2], q[3], q[4], q[5], X, Nn);
            store6<NT>(pos, nrm, (size_t)N, (size_t)v, X, Nn, NRM);
        }
    }
}

template <class T, bool NRM, bool NT, int RL>
static void launch_surface_t(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                             const SurfaceConfig& cfg, hipStream_t st)
{
    if (cfg.kind == 0) {
        const int n_col_tiles = (n_v + kBlock - 1) / kBlock;
        const int R = cfg.rows_per_block > 0 ? cfg.rows_per_block : 1;
        const long long grid = (long long)n_col_tiles * ((n_u + R - 1) / R);
        hipLaunchKernelGGL((k_surface_tiles<T, NRM, NT, RL>), dim3((unsigned)grid), dim3(kBlock), 0, st,
                           rows, prof, n_u, n_v, R, n_col_tiles, pos, nrm);
    } else {
        const long long N = (long long)n_u * n_v;
        const FastDiv dv = make_fastdiv(n_v);
        const int K = cfg.tile_vertices / kBlock;
        const unsigned grid = (unsigned)((N + cfg.tile_vertices - 1) / cfg.tile_vertices);
        switch (K) {
        case 1: hipLaunchKernelGGL((k_surface_linear<T, NRM, NT, 1, RL>), dim3(grid), dim3(kBlock), 0, st, rows, prof, n_u, n_v, dv, pos, nrm); break;
        case 2: hipLaunchKernelGGL((k_surface_linear<T, NRM, NT, 2, RL>), dim3(grid), dim3(kBlock), 0, st, rows, prof, n_u, n_v, dv, pos, nrm); break;
        case 4: hipLaunchKernelGGL((k_surface_linear<T, NRM, NT, 4, RL>), dim3(grid), dim3(kBlock), 0, st, rows, prof, n_u, n_v, dv, pos, nrm); break;
        default: hipLaunchKernelGGL((k_surface_linear<T, NRM, NT, 8, RL>), dim3(grid), dim3(kBlock), 0, st, rows, prof, n_u, n_v, dv, pos, nrm); break;
        }
    }
}

template <class T, int RL>
static void launch_surface_rl(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                              const SurfaceConfig& cfg, hipStream_t st)
{
    const bool wn = nrm != nullptr;
    if (cfg.nontemporal) {
        if (wn) launch_surface_t<T, true, true, RL>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
        else launch_surface_t<T, false, true, RL>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    } else {
        if (wn) launch_surface_t<T, true, false, RL>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
        else launch_surface_t<T, false, false, RL>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    }
}

template <class T>
hipError_t launch_surface(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                          const SurfaceConfig& cfg, hipStream_t st, bool ext)
{
    if (ext) launch_surface_rl<T, kRowExt>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    else launch_surface_rl<T, 16>(rows, prof, n_u, n_v, pos, nrm, cfg, st);
    return hipGetLastError();
}
template hipError_t launch_surface<float>(const float*, const float*, int, int, float*, float*,
                                          const SurfaceConfig&, hipStream_t, bool);
template hipError_t launch_surface<double>(const double*, const double*, int, int, double*, double*,
                                           const SurfaceConfig&, hipStream_t, bool);

}  // namespace sweep
