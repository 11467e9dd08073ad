// batched_kernels.hip -- a batch of independent sweeps in two launches.
//
// kb_frames   one block per sweep: its profile table, then the same three
//             frame passes as the single-sweep path (chunk products of the
//             step rotations, the carry scan, the row records), run
//             chunk after chunk inside the block.  Samples are recomputed in
//             the third pass instead of being stored.
// kb_surface  one block per tile of 256*K consecutive vertices of one sweep
//             (a host-built tile list covers every sweep), rows staged in
//             LDS, one vertex per lane per step, six plane stores.
//
// Both call the same device functions as the single-sweep kernels in the
// same order, so sweep k of a batch is bitwise identical to evaluating it
// alone.
#include "frame_common.hpp"
#include "surface_common.hpp"

namespace sweep {

struct ChunkState {
    int carry_lv;        // last sample with C' != 0 before this chunk (-1 if none)
    V3<double> d_carry;  // its C'
};

// This thread's step inputs for chunk b, plus its own C' and C''.  Contains
// barriers; called by every thread of the block.
__device__ StepInputs chunk_inputs(const DCurve& path, int n_u, int b, ChunkState& cs, V3<double> fb,
                                   double (*sx)[kChunk + 1], double (*sd)[kChunk + 1], int* lds_i,
                                   V3<double>& c1, V3<double>& c2)
{
    const int base = b * kChunk;
    const int i = base + threadIdx.x;
    V3<double> x0 = mk(0.0, 0.0, 0.0), d0 = x0;
    c2 = x0;
    if (i < n_u) {
        V3<double> o[3];
        sample_derivs_any<2>(path, i, n_u, o);
        x0 = o[0]; d0 = o[1]; c2 = o[2];
    }
    c1 = d0;
    sx[0][threadIdx.x] = x0.x; sx[1][threadIdx.x] = x0.y; sx[2][threadIdx.x] = x0.z;
    sd[0][threadIdx.x] = d0.x; sd[1][threadIdx.x] = d0.y; sd[2][threadIdx.x] = d0.z;
    if (threadIdx.x == 0 && base + kChunk < n_u) {
        V3<double> o[2];
        sample_derivs_any<1>(path, base + kChunk, n_u, o);
        sx[0][kChunk] = o[0].x; sx[1][kChunk] = o[0].y; sx[2][kChunk] = o[0].z;
        sd[0][kChunk] = o[1].x; sd[1][kChunk] = o[1].y; sd[2][kChunk] = o[1].z;
    }
    __syncthreads();
    const bool has_step = i + 1 < n_u;
    V3<double> x1 = x0, d1 = x0;
    if (has_step) {
        x1 = mk(sx[0][threadIdx.x + 1], sx[1][threadIdx.x + 1], sx[2][threadIdx.x + 1]);
        d1 = mk(sd[0][threadIdx.x + 1], sd[1][threadIdx.x + 1], sd[2][threadIdx.x + 1]);
    }
    const bool valid0 = i < n_u && dot(d0, d0) > 0.0;
    const bool valid1 = has_step && dot(d1, d1) > 0.0;
    int total;
    const int excl = block_exclusive_max(valid0 ? i : -1, lds_i, total);
    const int lv = max(cs.carry_lv, valid0 ? i : excl);
    V3<double> d_lv = d0;
    if (!valid0 && lv >= 0)
        d_lv = lv >= base ? mk(sd[0][lv - base], sd[1][lv - base], sd[2][lv - base]) : cs.d_carry;
    const StepInputs s = resolve_step(x0, d0, valid0, x1, d1, valid1, has_step, lv, d_lv, fb);
    if (total >= 0) {
        cs.carry_lv = total;
        cs.d_carry = mk(sd[0][total - base], sd[1][total - base], sd[2][total - base]);
    }
    __syncthreads();
    return s;
}

template <class F, class T>
__global__ __launch_bounds__(kBlock) void kb_frames(const BatchDesc* __restrict__ descs,
                                                    const double* __restrict__ path_ctrl,
                                                    const double* __restrict__ prof_ctrl,
                                                    const double* __restrict__ knots, InitialNormal n0, int reorth,
                                                    F* agg, F* r_in, T* __restrict__ rows, T* __restrict__ ptab)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    __shared__ double sx[3][kChunk + 1], sd[3][kChunk + 1];
    __shared__ double t0s[3];
    const BatchDesc d = descs[blockIdx.x];
    const DCurve path{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr,
                      d.n_path, d.p_path, 0, d.n_path};
    const DCurve prof{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr,
                      d.n_prof, d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof};
    T* ptab_k = ptab + 8 * d.ptab_off;
    for (int j = threadIdx.x; j < d.n_v; j += kBlock) write_profile<T>(prof, j, d.n_v, ptab_k);

    const int n_u = d.n_u;
    const int nc = (n_u + kChunk - 1) / kChunk;
    F* agg_k = agg + 9 * d.chunk_off;
    F* rin_k = r_in + 3 * d.chunk_off;
    const V3<double> fb = first_leg(path);
    ChunkState cs{-1, mk(0.0, 0.0, 0.0)};
    for (int b = 0; b < nc; ++b) {
        V3<double> c1, c2;
        const StepInputs s = chunk_inputs(path, n_u, b, cs, fb, sx, sd, lds_i, c1, c2);
        if (b == 0 && threadIdx.x == 0) { t0s[0] = s.t0.x; t0s[1] = s.t0.y; t0s[2] = s.t0.z; }
        M3<F> total;
        block_exclusive_product<F>(step_of<F>(s), lds_m, total);
        if (threadIdx.x < 9) agg_k[9 * (size_t)b + threadIdx.x] = total.m[threadIdx.x];
    }
    __threadfence_block();
    __syncthreads();
    carry_scan<F>(agg_k, nc, initial_normal(mk(t0s[0], t0s[1], t0s[2]), n0), rin_k, lds_m);
    __threadfence_block();
    __syncthreads();
    cs = ChunkState{-1, mk(0.0, 0.0, 0.0)};
    T* rows_k = rows + 16 * d.row_off;
    for (int b = 0; b < nc; ++b) {
        V3<double> c1, c2;
        const StepInputs s = chunk_inputs(path, n_u, b, cs, fb, sx, sd, lds_i, c1, c2);
        M3<F> total;
        const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m, total);
        const int i = b * kChunk + threadIdx.x;
        const F* rb = rin_k + 3 * (size_t)b;
        if (i < n_u) write_row<F, T>(s, ex, rb, c1, c2, reorth, rows_k + 16 * (size_t)i);
    }
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
    k.frames = (const void*)&kb_frames<F, T>;
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
