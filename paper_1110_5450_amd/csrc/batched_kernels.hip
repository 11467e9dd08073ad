// batched_kernels.hip -- a batch of independent sweeps, replayed as one HIP
// graph:
//
// kb_profile  one block per (sweep, chunk of 256 v-samples): profile tables.
// kb_prep     one block per (sweep, chunk of 256 u-samples), one launch per
//             path degree present (degree as a template parameter, so the
//             B-spline arrays stay in registers): samples, the chunk's last
//             valid sample and the ordered product of its step rotations (a
//             chunk whose first sample has C' = 0 is flagged).
// kb_carry    one block per sweep: products of its flagged chunks, then the
//             scan giving the normal entering each chunk.
// kb_apply    one block per (sweep, chunk), one launch per path degree: row
//             records.
// kb_surface  one block per tile of 256*K consecutive vertices of one sweep,
//             rows staged in LDS, one vertex per lane per step, six plane
//             stores.
//
// Samples are evaluated again in kb_apply instead of being stored.  Every
// step calls the same device functions as the single-sweep kernels in the
// same order (FP contraction off), so sweep k of a batch is bitwise identical
// to evaluating it alone.
#include "frame_common.hpp"
#include "surface_common.hpp"

namespace sweep {

__device__ __forceinline__ DCurve path_of(const BatchDesc& d, const double* path_ctrl, const double* knots)
{
    return DCurve{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr,
                  d.n_path, d.p_path, 0, d.n_path};
}
__device__ __forceinline__ DCurve prof_of(const BatchDesc& d, const double* prof_ctrl, const double* knots)
{
    return DCurve{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr,
                  d.n_prof, d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof};
}

struct ChunkLds {
    double sx[3][kChunk + 1];
    double sd[3][kChunk + 1];
    double d3[3];
    int ii[kWaves];
};

// This thread's step inputs for chunk b of a sweep, its own C' and C'', the
// chunk's last valid sample (`last`) and whether its first sample has
// C' != 0.  When the first sample has C' = 0 and chunk_lv (the last valid
// sample of each earlier chunk) is given, the tangent carried into the chunk
// is resolved from it; without chunk_lv the step inputs are not meaningful
// for such a chunk.  Contains barriers; called by every thread of the block.
template <int P>
__device__ StepInputs chunk_inputs(const DCurve& path, int n_u, int b, const int* chunk_lv, V3<double> fb,
                                   ChunkLds& L, V3<double>& c1, V3<double>& c2, int& last, bool& first_valid)
{
    const int base = b * kChunk;
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
    const V3<double> dfirst = mk(L.sd[0][0], L.sd[1][0], L.sd[2][0]);
    first_valid = dot(dfirst, dfirst) > 0.0;
    int carry_lv = -1;
    V3<double> d_carry = mk(0.0, 0.0, 0.0);
    int total;
    if (b > 0 && !first_valid && chunk_lv) {
        int c = -1;
        for (int k = threadIdx.x; k < b; k += kBlock) c = max(c, chunk_lv[k]);
        block_exclusive_max(c, L.ii, total);
        carry_lv = total;
        if (carry_lv >= 0) {
            if (threadIdx.x == 0) {
                V3<double> o[2];
                sample_derivs<P, 1>(path, carry_lv, n_u, o);
                L.d3[0] = o[1].x; L.d3[1] = o[1].y; L.d3[2] = o[1].z;
            }
            __syncthreads();
            d_carry = mk(L.d3[0], L.d3[1], L.d3[2]);
        }
    }
    const bool has_step = i + 1 < n_u;
    V3<double> x1 = x0, d1 = x0;
    if (has_step) {
        x1 = mk(L.sx[0][threadIdx.x + 1], L.sx[1][threadIdx.x + 1], L.sx[2][threadIdx.x + 1]);
        d1 = mk(L.sd[0][threadIdx.x + 1], L.sd[1][threadIdx.x + 1], L.sd[2][threadIdx.x + 1]);
    }
    const bool valid0 = i < n_u && dot(d0, d0) > 0.0;
    const bool valid1 = has_step && dot(d1, d1) > 0.0;
    const int excl = block_exclusive_max(valid0 ? i : -1, L.ii, total);
    last = total;
    const int lv = max(carry_lv, valid0 ? i : excl);
    V3<double> d_lv = d0;
    if (!valid0 && lv >= 0)
        d_lv = lv >= base ? mk(L.sd[0][lv - base], L.sd[1][lv - base], L.sd[2][lv - base]) : d_carry;
    const StepInputs s = resolve_step(x0, d0, valid0, x1, d1, valid1, has_step, lv, d_lv, fb);
    __syncthreads();
    return s;
}

// Profile tables: one block per (sweep, chunk of 256 v-samples).
template <class T>
__global__ __launch_bounds__(kBlock) void kb_profile(const BatchDesc* __restrict__ descs,
                                                     const int2* __restrict__ vchunks,
                                                     const double* __restrict__ prof_ctrl,
                                                     const double* __restrict__ knots, T* __restrict__ ptab)
{
    const int2 vc = vchunks[blockIdx.x];
    const BatchDesc d = descs[vc.x];
    const int j = vc.y * kBlock + threadIdx.x;
    if (j < d.n_v) write_profile<T>(prof_of(d, prof_ctrl, knots), j, d.n_v, ptab + 8 * d.ptab_off);
}

// One block per (sweep, chunk) of the sweeps whose path has degree P.
template <int P, class F>
__global__ __launch_bounds__(kBlock) void kb_prep(const BatchDesc* __restrict__ descs, const int2* __restrict__ chunks,
                                                  const double* __restrict__ path_ctrl,
                                                  const double* __restrict__ knots, F* __restrict__ agg,
                                                  int* __restrict__ chunk_lv, int* __restrict__ chunk_fix)
{
    __shared__ ChunkLds L;
    __shared__ M3<F> lds_m[kWaves];
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const DCurve path = path_of(d, path_ctrl, knots);
    const int b = ch.y;
    V3<double> c1, c2;
    int last;
    bool first_valid;
    const StepInputs s = chunk_inputs<P>(path, d.n_u, b, nullptr, first_leg(path), L, c1, c2, last, first_valid);
    const size_t c = (size_t)d.chunk_off + b;
    if (threadIdx.x == 0) {
        chunk_lv[c] = last;
        chunk_fix[c] = (b > 0 && !first_valid) ? 1 : 0;
    }
    if (b > 0 && !first_valid) return;   // formed by kb_carry (block-uniform)
    M3<F> prod;
    block_exclusive_product<F>(step_of<F>(s), lds_m, prod);
    if (threadIdx.x < 9) agg[9 * c + threadIdx.x] = prod.m[threadIdx.x];
}

// One block per sweep: flagged chunk products, then the carry scan.
template <class F>
__global__ __launch_bounds__(kBlock) void kb_carry(const BatchDesc* __restrict__ descs,
                                                   const double* __restrict__ path_ctrl,
                                                   const double* __restrict__ knots, InitialNormal n0, F* agg,
                                                   const int* __restrict__ chunk_lv,
                                                   const int* __restrict__ chunk_fix, F* __restrict__ r_in)
{
    __shared__ ChunkLds L;
    __shared__ M3<F> lds_m[kWaves];
    const BatchDesc d = descs[blockIdx.x];
    const DCurve path = path_of(d, path_ctrl, knots);
    const int nc = (d.n_u + kChunk - 1) / kChunk;
    F* agg_k = agg + 9 * d.chunk_off;
    const int* lv_k = chunk_lv + d.chunk_off;
    const int* fix_k = chunk_fix + d.chunk_off;
    const V3<double> fb = first_leg(path);
    for (int b = 1; b < nc; ++b) {
        if (!fix_k[b]) continue;   // uniform
        V3<double> c1, c2;
        int last;
        bool first_valid;
        StepInputs s;
        switch (path.p) {
        case 1: s = chunk_inputs<1>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        case 2: s = chunk_inputs<2>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        case 3: s = chunk_inputs<3>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        case 4: s = chunk_inputs<4>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        case 5: s = chunk_inputs<5>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        case 6: s = chunk_inputs<6>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        default: s = chunk_inputs<7>(path, d.n_u, b, lv_k, fb, L, c1, c2, last, first_valid); break;
        }
        M3<F> prod;
        block_exclusive_product<F>(step_of<F>(s), lds_m, prod);
        if (threadIdx.x < 9) agg_k[9 * (size_t)b + threadIdx.x] = prod.m[threadIdx.x];
        __threadfence_block();
        __syncthreads();
    }
    // resolved t_0
    if (threadIdx.x == 0) {
        V3<double> o[2];
        sample_derivs_any<1>(path, 0, d.n_u, o);
        L.d3[0] = o[1].x; L.d3[1] = o[1].y; L.d3[2] = o[1].z;
    }
    __syncthreads();
    const V3<double> d0 = mk(L.d3[0], L.d3[1], L.d3[2]);
    const V3<double> t0 = dot(d0, d0) > 0.0 ? unit_of(d0) : fb;
    carry_scan<F>(agg_k, nc, initial_normal(t0, n0), r_in + 3 * d.chunk_off, lds_m);
}

template <int P, class F, class T>
__global__ __launch_bounds__(kBlock) void kb_apply(const BatchDesc* __restrict__ descs,
                                                   const int2* __restrict__ chunks,
                                                   const double* __restrict__ path_ctrl,
                                                   const double* __restrict__ knots, int reorth,
                                                   const int* __restrict__ chunk_lv, const F* __restrict__ r_in,
                                                   T* __restrict__ rows)
{
    __shared__ ChunkLds L;
    __shared__ M3<F> lds_m[kWaves];
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const DCurve path = path_of(d, path_ctrl, knots);
    const int b = ch.y;
    V3<double> c1, c2;
    int last;
    bool first_valid;
    const StepInputs s = chunk_inputs<P>(path, d.n_u, b, chunk_lv + d.chunk_off, first_leg(path), L, c1, c2, last,
                                         first_valid);
    M3<F> total;
    const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m, total);
    const int i = b * kChunk + threadIdx.x;
    if (i < d.n_u)
        write_row<F, T>(s, ex, r_in + 3 * ((size_t)d.chunk_off + b), c1, c2, reorth,
                        rows + 16 * ((size_t)d.row_off + i));
}

constexpr int kBatchK = 4;   // vertices per lane in the batched surface kernel

template <class T, bool NRM, bool NT>
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
    const long long vlast = min(N, v0 + kBlock * kBatchK) - 1;
    const T* rows_k = rows + 16 * d.row_off;
    const int ilo = fdiv((unsigned)v0, dv);
    const int nrow = fdiv((unsigned)vlast, dv) - ilo + 1;
    const bool staged = nrow <= kMaxLdsRows;
    if (staged)
        for (int e = threadIdx.x; e < nrow * 16; e += kBlock) lrow[e] = rows_k[16 * (size_t)ilo + e];
    __syncthreads();
    const T* ptab_k = ptab + 8 * d.ptab_off;
    T* pos_k = pos + 3 * d.out_off;
    T* nrm_k = NRM ? nrm + 3 * d.out_off : nrm;
#pragma unroll
    for (int k = 0; k < kBatchK; ++k) {
        const long long v = v0 + threadIdx.x + k * kBlock;
        if (v < N) {
            const int i = fdiv((unsigned)v, dv);
            const int j = (int)v - i * d.n_v;
            const T* q = ptab_k + 8 * (size_t)j;
            const T* row = staged ? lrow + 16 * (i - ilo) : rows_k + 16 * (size_t)i;
            T X[3], Nn[3];
            vertex<T>(row, q[0], q[1], q[2], q[3], q[4], q[5], X, Nn);
            store6<NT>(pos_k, nrm_k, (size_t)N, (size_t)v, X, Nn, NRM);
        }
    }
}

int batched_tile_vertices() { return kBlock * kBatchK; }

template <class F, class T>
static BatchedKernels pick(bool nrm, bool nt)
{
    BatchedKernels k;
    k.profile = (const void*)&kb_profile<T>;
    k.prep[0] = k.apply[0] = nullptr;
#define SWEEP_DEG(P) \
    k.prep[P] = (const void*)&kb_prep<P, F>; \
    k.apply[P] = (const void*)&kb_apply<P, F, T>;
    SWEEP_DEG(1) SWEEP_DEG(2) SWEEP_DEG(3) SWEEP_DEG(4) SWEEP_DEG(5) SWEEP_DEG(6) SWEEP_DEG(7)
#undef SWEEP_DEG
    k.carry = (const void*)&kb_carry<F>;
    if (nrm) k.surface = nt ? (const void*)&kb_surface<T, true, true> : (const void*)&kb_surface<T, true, false>;
    else k.surface = nt ? (const void*)&kb_surface<T, false, true> : (const void*)&kb_surface<T, false, false>;
    return k;
}

BatchedKernels batched_kernels(bool f64, bool t64, bool nrm, bool nontemporal)
{
    if (f64) return t64 ? pick<double, double>(nrm, nontemporal) : pick<double, float>(nrm, nontemporal);
    return t64 ? pick<float, double>(nrm, nontemporal) : pick<float, float>(nrm, nontemporal);
}

}  // namespace sweep
