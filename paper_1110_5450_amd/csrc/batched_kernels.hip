// batched_kernels.hip -- a batch of independent sweeps, replayed as one HIP
// graph:
//
// kb_profile  one block per (sweep, chunk of 256 v-samples): profile tables.
// kb_frame    one block per sweep, one launch per path degree present (the
//             degree is a template parameter, so the B-spline arrays stay in
//             registers); sweeps are listed longest first.  The block walks
//             its sweep's chunks of 256 u-samples in order: samples, step
//             rotations, the block's exclusive product scan, row records,
//             then the normal entering the next chunk (the chunk's total
//             product applied to the normal entering it) and the last sample
//             with C' != 0 are carried in registers.  Every sample is
//             evaluated once and no cross-block carry is needed.
// kb_surface  one block per tile of 256*K (K = 1, 2, 4, 8) consecutive
//             vertices of one sweep, rows staged in LDS, one vertex per lane
//             per step, six plane stores.
//
// The per-sample and per-chunk steps call the same device functions as the
// single-sweep kernels in the same order (FP contraction off): a sweep of at
// most one chunk is bitwise identical to evaluating it alone; longer sweeps
// differ only in how the chunk products are associated (sequential here, a
// tree scan there), i.e. by rounding.
#include "frame_common.hpp"
#include "surface_common.hpp"

namespace sweep {

__device__ __forceinline__ DCurve path_of(const BatchDesc& d, const double* path_ctrl, const double* path_w,
                                          const double* knots)
{
    return DCurve{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr,
                  d.n_path, d.p_path, 0, d.n_path, path_w ? path_w + d.path_ctrl_off : nullptr};
}
__device__ __forceinline__ DCurve prof_of(const BatchDesc& d, const double* prof_ctrl, const double* prof_w,
                                          const double* knots)
{
    return DCurve{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr,
                  d.n_prof, d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof,
                  prof_w ? prof_w + d.prof_ctrl_off : nullptr};
}

struct ChunkLds {
    double sx[3][kChunk + 1];
    double sd[3][kChunk + 1];
    double d3[3];
    int ii[kWaves];
};

// This thread's step inputs for the chunk starting at `base`, its own C' and
// C'', given the last sample before the chunk with C' != 0 (carry_lv, -1 if
// none) and its C' (d_carry).  Returns in `last` / `d_last` the last sample
// up to the chunk's end with C' != 0 and its C' (the carry for the next
// chunk).  Contains barriers; called by every thread of the block.
template <int P>
__device__ StepInputs seq_chunk_inputs(const DCurve& path, int n_u, int base, int carry_lv, V3<double> d_carry,
                                       V3<double> fb, ChunkLds& L, V3<double>& c1, V3<double>& c2, int& last,
                                       V3<double>& d_last)
{
    const int i = base + threadIdx.x;
    V3<double> x0 = mk(0.0, 0.0, 0.0), d0 = x0;
    c2 = x0;
    if (i < n_u) {
        V3<double> o[3];
        sample_derivs<P, 2>(path, i, n_u, o);
        x0 = o[0]; d0 = o[1]; c2 = o[2];
    }
    c1 = d0;
    L.sx[0][threadIdx.x] = x0.x; L.sx[1][threadIdx.x] = x0.y; L.sx[2][threadIdx.x] = x0.z;
    L.sd[0][threadIdx.x] = d0.x; L.sd[1][threadIdx.x] = d0.y; L.sd[2][threadIdx.x] = d0.z;
    if (threadIdx.x == 0 && base + kChunk < n_u) {
        V3<double> o[2];
        sample_derivs<P, 1>(path, base + kChunk, n_u, o);
        L.sx[0][kChunk] = o[0].x; L.sx[1][kChunk] = o[0].y; L.sx[2][kChunk] = o[0].z;
        L.sd[0][kChunk] = o[1].x; L.sd[1][kChunk] = o[1].y; L.sd[2][kChunk] = o[1].z;
    }
    __syncthreads();
    const bool has_step = i + 1 < n_u;
    V3<double> x1 = x0, d1 = x0;
    if (has_step) {
        x1 = mk(L.sx[0][threadIdx.x + 1], L.sx[1][threadIdx.x + 1], L.sx[2][threadIdx.x + 1]);
        d1 = mk(L.sd[0][threadIdx.x + 1], L.sd[1][threadIdx.x + 1], L.sd[2][threadIdx.x + 1]);
    }
    const bool valid0 = i < n_u && dot(d0, d0) > 0.0;
    const bool valid1 = has_step && dot(d1, d1) > 0.0;
    int total;
    const int excl = block_exclusive_max(valid0 ? i : -1, L.ii, total);
    const int lv = max(carry_lv, valid0 ? i : excl);
    V3<double> d_lv = d0;
    if (!valid0 && lv >= 0)
        d_lv = lv >= base ? mk(L.sd[0][lv - base], L.sd[1][lv - base], L.sd[2][lv - base]) : d_carry;
    const StepInputs s = resolve_step(x0, d0, valid0, x1, d1, valid1, has_step, lv, d_lv, fb);
    if (total >= 0) {
        last = total;
        d_last = mk(L.sd[0][total - base], L.sd[1][total - base], L.sd[2][total - base]);
    } else {
        last = carry_lv;
        d_last = d_carry;
    }
    __syncthreads();
    return s;
}

// Profile tables: one block per (sweep, chunk of 256 v-samples).
template <class T>
__global__ __launch_bounds__(kBlock) void kb_profile(const BatchDesc* __restrict__ descs,
                                                     const int2* __restrict__ vchunks,
                                                     const double* __restrict__ prof_ctrl,
                                                     const double* __restrict__ prof_w,
                                                     const double* __restrict__ knots, T* __restrict__ ptab)
{
    const int2 vc = vchunks[blockIdx.x];
    const BatchDesc d = descs[vc.x];
    const int j = vc.y * kBlock + threadIdx.x;
    if (j < d.n_v) write_profile<T>(prof_of(d, prof_ctrl, prof_w, knots), j, d.n_v, ptab + 8 * d.ptab_off);
}

// Row records of the sweeps whose path has degree P: one block per sweep.
template <int P, class F, class T>
__global__ __launch_bounds__(kBlock) void kb_frame(const BatchDesc* __restrict__ descs,
                                                   const int* __restrict__ sweeps,
                                                   const double* __restrict__ path_ctrl,
                                                   const double* __restrict__ path_w,
                                                   const double* __restrict__ knots, InitialNormal n0, int reorth,
                                                   T* __restrict__ rows)
{
    __shared__ ChunkLds L;
    __shared__ M3<F> lds_m[kWaves];
    const BatchDesc d = descs[sweeps[blockIdx.x]];
    const DCurve path = path_of(d, path_ctrl, path_w, knots);
    const V3<double> fb = first_leg(path);
    const int n_u = d.n_u;
    T* rows_k = rows + 16 * (size_t)d.row_off;
    int lv = -1;
    V3<double> d_lv = mk(0.0, 0.0, 0.0);
    F rin[3];
    for (int base = 0; base < n_u; base += kChunk) {
        V3<double> c1, c2, d_last;
        int last;
        const StepInputs s = seq_chunk_inputs<P>(path, n_u, base, lv, d_lv, fb, L, c1, c2, last, d_last);
        lv = last;
        d_lv = d_last;
        if (base == 0) {
            // r_0 from the resolved t_0 (sample 0 is thread 0's)
            if (threadIdx.x == 0) { L.d3[0] = s.t0.x; L.d3[1] = s.t0.y; L.d3[2] = s.t0.z; }
            __syncthreads();
            const V3<F> r0 = cvt<F>(initial_normal(mk(L.d3[0], L.d3[1], L.d3[2]), n0));
            rin[0] = r0.x; rin[1] = r0.y; rin[2] = r0.z;
        }
        M3<F> total;
        const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m, total);
        const int i = base + threadIdx.x;
        if (i < n_u) write_row<F, T>(s, ex, rin, c1, c2, reorth, rows_k + 16 * (size_t)i);
        const V3<F> rn = apply(total, mk(rin[0], rin[1], rin[2]));
        rin[0] = rn.x; rin[1] = rn.y; rin[2] = rn.z;
    }
}

// K = vertices per lane (tile of 256*K vertices per block).
template <class T, bool NRM, bool NT, int K>
__global__ __launch_bounds__(kBlock) void kb_surface(const BatchDesc* __restrict__ descs,
                                                     const int2* __restrict__ tiles, const T* __restrict__ rows,
                                                     const T* __restrict__ ptab, T* __restrict__ pos,
                                                     T* __restrict__ nrm)
{
    __shared__ T lrow[kMaxLdsRows * 16];
    const int2 tl = tiles[blockIdx.x];
    const BatchDesc d = descs[tl.x];
    const FastDiv dv{d.fd_m, d.fd_shift, d.n_v};
    const long long N = (long long)d.n_u * (long long)d.n_v;
    const long long v0 = tl.y;
    const long long vlast = min(N, v0 + kBlock * K) - 1;
    const T* rows_k = rows + 16 * d.row_off;
    const int ilo = fdiv((unsigned)v0, dv);
    const int nrow = fdiv((unsigned)vlast, dv) - ilo + 1;
    const bool staged = nrow <= kMaxLdsRows;
    if (staged)
        for (int e = threadIdx.x; e < nrow * 16; e += kBlock) lrow[e] = rows_k[16 * (size_t)ilo + e];
    __syncthreads();
    const T* ptab_k = ptab + 8 * d.ptab_off;
    T* pos_k = pos + d.out_off;
    T* nrm_k = NRM ? nrm + d.out_off : nrm;
    // The profile records of all K vertices are loaded before the first
    // store: on this ISA the vector-memory counter also counts stores, so a
    // load issued after a store would wait for it.  Row records come from
    // LDS (or, for a tile of more than kMaxLdsRows rows, from global memory).
    T qv[K][6];
    int vi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long v = v0 + threadIdx.x + k * kBlock;
        vi[k] = 0;
#pragma unroll
        for (int e = 0; e < 6; ++e) qv[k][e] = T(0);
        if (v < N) {
            const int i = fdiv((unsigned)v, dv);
            const int j = (int)v - i * d.n_v;
            vi[k] = i;
            const T* q = ptab_k + 8 * (size_t)j;
#pragma unroll
            for (int e = 0; e < 6; ++e) qv[k][e] = q[e];
        }
    }
    // the sweep's last tile also covers the plane padding [N, plane), which
    // is zeroed (plane <= N rounded up to the tile size).  Two copies of the
    // row reads (block-uniform choice), so that the staged one reads LDS only.
    // All K vertices are formed before the first store, for the same reason.
    T X[K][3], Nn[K][3];
    auto form = [&](const T* base, int row0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) X[k][c] = Nn[k][c] = T(0);
            if (v0 + threadIdx.x + k * kBlock < N)
                vertex<T>(base + 16 * (size_t)(vi[k] - row0), qv[k][0], qv[k][1], qv[k][2], qv[k][3], qv[k][4],
                          qv[k][5], X[k], Nn[k]);
        }
    };
    if (staged) form(lrow, ilo);
    else form(rows_k, 0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long v = v0 + threadIdx.x + k * kBlock;
        if (v < d.plane) store6<NT>(pos_k, nrm_k, (size_t)d.plane, (size_t)v, X[k], Nn[k], NRM);
    }
}

template <class T, bool NRM, bool NT>
static const void* surface_for(int K)
{
    switch (K) {
    case 1: return (const void*)&kb_surface<T, NRM, NT, 1>;
    case 2: return (const void*)&kb_surface<T, NRM, NT, 2>;
    case 4: return (const void*)&kb_surface<T, NRM, NT, 4>;
    default: return (const void*)&kb_surface<T, NRM, NT, 8>;
    }
}

template <class F, class T>
static BatchedKernels pick(bool nrm, bool nt, int K)
{
    BatchedKernels k;
    k.profile = (const void*)&kb_profile<T>;
    k.frame[0] = nullptr;
#define SWEEP_DEG(P) k.frame[P] = (const void*)&kb_frame<P, F, T>;
    SWEEP_DEG(1) SWEEP_DEG(2) SWEEP_DEG(3) SWEEP_DEG(4) SWEEP_DEG(5) SWEEP_DEG(6) SWEEP_DEG(7)
#undef SWEEP_DEG
    if (nrm) k.surface = nt ? surface_for<T, true, true>(K) : surface_for<T, true, false>(K);
    else k.surface = nt ? surface_for<T, false, true>(K) : surface_for<T, false, false>(K);
    return k;
}

BatchedKernels batched_kernels(bool f64, bool t64, bool nrm, bool nontemporal, int tile_vertices)
{
    const int K = tile_vertices / kBlock;
    if (f64) return t64 ? pick<double, double>(nrm, nontemporal, K) : pick<double, float>(nrm, nontemporal, K);
    return t64 ? pick<float, double>(nrm, nontemporal, K) : pick<float, float>(nrm, nontemporal, K);
}

}  // namespace sweep
