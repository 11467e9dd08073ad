// frame_kernels.hip -- curve sampling and the rotation-minimizing frame of a
// single sweep as a parallel prefix product of 3x3 rotations, in three
// launches:
//
// k_prep          per chunk of kChunk u-samples: C, C', C'' (FP64, SoA
//                 planes), the last sample with C' != 0, tangents (a sample
//                 with C' = 0 takes the tangent of the last sample before it
//                 with C' != 0), step rotations M_i and their ordered product
//                 A_b.  A chunk whose first sample has C' = 0 needs the
//                 tangent of an earlier chunk: it is flagged and its product
//                 is formed by k_frame_carry.  Extra blocks write the profile
//                 table (S, S' in the output precision).
// k_frame_carry   one block: products of flagged chunks, then the scan of the
//                 A_b giving the normal entering each chunk,
//                 r_in[b] = (A_{b-1} ... A_0) r_0.  (A separate launch: a
//                 last-block hand-off inside k_prep would need a device-scope
//                 fence per block, whose L2 write-back across the eight XCDs
//                 measured 37 us at 256 chunks and 360 us at 4096.)
// k_frame_apply   per chunk: block exclusive product of the M_i applied to
//                 r_in[b], re-orthonormalisation, and the row table
//                 (x, r, s, t, |C'|, a, b) in the output precision.
//
// k_frame_apply rebuilds the step rotations from the same inputs with the
// same code as k_prep, so both see bitwise identical M_i.
//
// With at most kBlock chunks (and no frame mode or law), k_frame_apply_fused
// replaces k_frame_carry + k_frame_apply: block b forms its own entry normal
// as the ordered block product of the chunk products below it, applied to
// r_0 (one launch fewer; the chunk products are combined in a tree instead
// of the carry's scan, the same to rounding).
#include "frame_common.hpp"

namespace sweep {

// smp layout: plane c (0..8 = x, C', C'') of n_u doubles.
__device__ __forceinline__ V3<double> smp_get(const double* __restrict__ smp, size_t n_u, int plane, int i)
{
    return {smp[(size_t)(3 * plane) * n_u + i], smp[(size_t)(3 * plane + 1) * n_u + i],
            smp[(size_t)(3 * plane + 2) * n_u + i]};
}

// Step inputs of this thread's sample i = b*kChunk + tid from the sample
// planes.  Called by every thread of the block (contains barriers).
__device__ StepInputs load_step_inputs(const double* __restrict__ smp, int n_u, const int* __restrict__ chunk_lv,
                                       const double* __restrict__ fallback_t, int* lds_i, int b)
{
    const size_t nu = (size_t)n_u;
    const int base = b * kChunk;
    const int i = base + threadIdx.x;
    int total;
    // The last sample with C' != 0 before this chunk matters only when the
    // chunk's first sample has C' = 0 (a block-uniform test).
    int carry = -1;
    const V3<double> dfirst = smp_get(smp, nu, 1, base);
    if (b > 0 && !(dot(dfirst, dfirst) > 0.0)) {
        for (int k = threadIdx.x; k < b; k += kBlock) carry = max(carry, chunk_lv[k]);
        block_exclusive_max(carry, lds_i, total);
        carry = total;
    }
    const bool has_step = i + 1 < n_u;
    V3<double> x0 = mk(0.0, 0.0, 0.0), d0 = x0, x1 = x0, d1 = x0;
    if (i < n_u) { x0 = smp_get(smp, nu, 0, i); d0 = smp_get(smp, nu, 1, i); }
    if (has_step) { x1 = smp_get(smp, nu, 0, i + 1); d1 = smp_get(smp, nu, 1, i + 1); }
    const bool valid0 = i < n_u && dot(d0, d0) > 0.0;
    const bool valid1 = has_step && dot(d1, d1) > 0.0;
    const int excl = block_exclusive_max(valid0 ? i : -1, lds_i, total);
    const int lv = max(carry, valid0 ? i : excl);
    const V3<double> d_lv = (!valid0 && lv >= 0) ? smp_get(smp, nu, 1, lv) : d0;
    return resolve_step(x0, d0, valid0, x1, d1, valid1, has_step, lv, d_lv,
                        mk(fallback_t[0], fallback_t[1], fallback_t[2]));
}

// Blocks [0, ncu): path samples and chunk products; blocks [ncu, ncu + ncv):
// profile table.
template <int P, class F, class T>
__global__ __launch_bounds__(kBlock) void k_prep(DCurve path, int n_u, DCurve prof, int n_v, int ncu,
                                                 double* __restrict__ smp, int* __restrict__ chunk_lv,
                                                 int* __restrict__ chunk_fix, double* __restrict__ fallback_t,
                                                 F* __restrict__ agg, T* __restrict__ ptab)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    __shared__ double sx[3][kChunk + 1], sd[3][kChunk + 1];
    if ((int)blockIdx.x >= ncu) {
        const int j = ((int)blockIdx.x - ncu) * kBlock + threadIdx.x;
        if (j < n_v) write_profile<T>(prof, j, n_v, ptab);
        return;
    }
    const size_t nu = (size_t)n_u;
    const int b = blockIdx.x;
    const int base = b * kChunk;
    const int i = base + threadIdx.x;
    V3<double> x0 = mk(0.0, 0.0, 0.0), d0 = x0;
    if (i < n_u) {
        V3<double> o[3];
        sample_derivs<P, 2>(path, i, n_u, o);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            smp[(size_t)(3 * d) * nu + i] = o[d].x;
            smp[(size_t)(3 * d + 1) * nu + i] = o[d].y;
            smp[(size_t)(3 * d + 2) * nu + i] = o[d].z;
        }
        x0 = o[0];
        d0 = o[1];
    }
    sx[0][threadIdx.x] = x0.x; sx[1][threadIdx.x] = x0.y; sx[2][threadIdx.x] = x0.z;
    sd[0][threadIdx.x] = d0.x; sd[1][threadIdx.x] = d0.y; sd[2][threadIdx.x] = d0.z;
    if (threadIdx.x == 0 && base + kChunk < n_u) {
        // first sample of the next chunk (also written by that chunk's block)
        V3<double> o[2];
        sample_derivs<P, 1>(path, base + kChunk, n_u, o);
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
    const bool first_valid = dot(mk(sd[0][0], sd[1][0], sd[2][0]), mk(sd[0][0], sd[1][0], sd[2][0])) > 0.0;
    if (threadIdx.x == 0) {
        chunk_lv[b] = total;
        chunk_fix[b] = (b > 0 && !first_valid) ? 1 : 0;
    }
    const V3<double> fb = first_leg(path);
    if (b == 0 && threadIdx.x == 0) {
        // used only when C'(u_0) = 0
        fallback_t[0] = fb.x; fallback_t[1] = fb.y; fallback_t[2] = fb.z;
    }
    if (b > 0 && !first_valid) return;   // product formed by k_frame_carry (block-uniform)
    const int lv = valid0 ? i : excl;
    V3<double> d_lv = d0;
    if (!valid0 && lv >= 0) d_lv = mk(sd[0][lv - base], sd[1][lv - base], sd[2][lv - base]);
    const StepInputs s = resolve_step(x0, d0, valid0, x1, d1, valid1, has_step, lv, d_lv, fb);
    const M3<F> prod = block_product<F>(step_of<F>(s), lds_m);
    if (threadIdx.x < 9) agg[9 * (size_t)b + threadIdx.x] = prod.m[threadIdx.x];
}

// One block: products of the flagged chunks (first sample with C' = 0), then
// r_in[c] = (A_{c-1} ... A_0) r_0 for every chunk.
template <class F>
__global__ __launch_bounds__(kBlock) void k_frame_carry(F* __restrict__ agg, int n_chunks,
                                                        const double* __restrict__ smp, int n_u,
                                                        const int* __restrict__ chunk_lv,
                                                        const int* __restrict__ chunk_fix,
                                                        const double* __restrict__ fallback_t, InitialNormal n0,
                                                        F* __restrict__ r_in)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    // any flagged chunk at all?  one strided pass and one block reduction
    int any = -1;
    for (int c = threadIdx.x; c < n_chunks; c += kBlock) any = chunk_fix[c] ? c : any;
    int last_flagged;
    block_exclusive_max(any, lds_i, last_flagged);
    for (int base = 0; base <= last_flagged; base += kBlock) {   // uniform; skipped when none
        const int c = base + threadIdx.x;
        int total;
        block_exclusive_max(c < n_chunks && chunk_fix[c] ? c : -1, lds_i, total);
        if (total < 0) continue;   // no flagged chunk in this range (uniform)
        for (int b = base; b < min(n_chunks, base + kBlock); ++b) {
            if (!chunk_fix[b]) continue;
            const StepInputs s = load_step_inputs(smp, n_u, chunk_lv, fallback_t, lds_i, b);
            const M3<F> prod = block_product<F>(step_of<F>(s), lds_m);
            if (threadIdx.x < 9) agg[9 * (size_t)b + threadIdx.x] = prod.m[threadIdx.x];
            __threadfence_block();
            __syncthreads();
        }
    }
    const V3<double> d = smp_get(smp, (size_t)n_u, 1, 0);
    const V3<double> t0 = dot(d, d) > 0.0 ? unit_of(d) : mk(fallback_t[0], fallback_t[1], fallback_t[2]);
    carry_scan<F>(agg, n_chunks, initial_normal(t0, n0), r_in, lds_m);
}

template <class F, class T>
__global__ __launch_bounds__(kBlock) void k_frame_apply(const double* __restrict__ smp, int n_u,
                                                        const int* __restrict__ chunk_lv,
                                                        const double* __restrict__ fallback_t,
                                                        const F* __restrict__ r_in, int reorth,
                                                        T* __restrict__ rows)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    const size_t nu = (size_t)n_u;
    const StepInputs s = load_step_inputs(smp, n_u, chunk_lv, fallback_t, lds_i, blockIdx.x);
    const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m);
    const int i = blockIdx.x * kChunk + threadIdx.x;
    if (i >= n_u) return;
    write_row<F, T>(s, ex, r_in + 3 * (size_t)blockIdx.x, smp_get(smp, nu, 1, i), smp_get(smp, nu, 2, i), reorth,
                    rows + 16 * (size_t)i);
}

// k_frame_apply without k_frame_carry, for at most kBlock chunks: thread c
// holds the product A_c of chunk c < b (identity above); the products of
// chunks whose first sample has C' = 0 (not formed by k_prep) are formed
// here, as k_frame_carry does; their ordered block product applied to r_0 is
// the block's entry normal.
template <class F, class T>
__global__ __launch_bounds__(kBlock) void k_frame_apply_fused(const double* __restrict__ smp, int n_u,
                                                              const int* __restrict__ chunk_lv,
                                                              const int* __restrict__ chunk_fix,
                                                              const double* __restrict__ fallback_t,
                                                              const F* __restrict__ agg, InitialNormal n0, int reorth,
                                                              T* __restrict__ rows)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    __shared__ M3<F> lds_fix;
    __shared__ int lflag[kBlock];
    __shared__ F lds_r[3];
    const size_t nu = (size_t)n_u;
    const int b = blockIdx.x, c = threadIdx.x;
    M3<F> A = ident<F>();
    int flagged = 0;
    if (c < b) {
        flagged = chunk_fix[c];
        if (!flagged) {
#pragma unroll
            for (int e = 0; e < 9; ++e) A.m[e] = agg[9 * (size_t)c + e];
        }
    }
    lflag[c] = flagged;
    int last_flagged;
    block_exclusive_max(flagged ? c : -1, lds_i, last_flagged);   // also orders lflag
    for (int f = 1; f <= last_flagged; ++f) {   // uniform; skipped when none
        if (!lflag[f]) continue;
        const StepInputs sf = load_step_inputs(smp, n_u, chunk_lv, fallback_t, lds_i, f);
        const M3<F> prod = block_product<F>(step_of<F>(sf), lds_m);
        if (threadIdx.x == 0) lds_fix = prod;
        __syncthreads();
        if (c == f) A = lds_fix;
        __syncthreads();
    }
    const M3<F> P = block_product<F>(A, lds_m);   // A_{b-1} ... A_0, valid in wave 0
    if (threadIdx.x == 0) {
        const V3<double> d = smp_get(smp, nu, 1, 0);
        const V3<double> t0 = dot(d, d) > 0.0 ? unit_of(d) : mk(fallback_t[0], fallback_t[1], fallback_t[2]);
        const V3<F> r = apply(P, cvt<F>(initial_normal(t0, n0)));
        lds_r[0] = r.x; lds_r[1] = r.y; lds_r[2] = r.z;
    }
    __syncthreads();
    const F rin[3] = {lds_r[0], lds_r[1], lds_r[2]};
    const StepInputs s = load_step_inputs(smp, n_u, chunk_lv, fallback_t, lds_i, b);
    const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m);
    const int i = b * kChunk + threadIdx.x;
    if (i >= n_u) return;
    write_row<F, T>(s, ex, rin, smp_get(smp, nu, 1, i), smp_get(smp, nu, 2, i), reorth, rows + 16 * (size_t)i);
}

// Extended row records (Frenet frame mode and/or a sweep law): the same
// block scan for the rotation-minimizing frame; the Frenet mode replaces r by
// the principal normal and needs the third derivative of the path, which is
// evaluated here (the samples hold x, C', C'' only).
template <class F, class T>
__global__ __launch_bounds__(kBlock) void k_frame_apply_ext(const double* __restrict__ smp, int n_u,
                                                            const int* __restrict__ chunk_lv,
                                                            const double* __restrict__ fallback_t,
                                                            const F* __restrict__ r_in, int reorth, DCurve path,
                                                            int frenet, DCurve law, int has_law, double du_scale,
                                                            T* __restrict__ rows)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    const size_t nu = (size_t)n_u;
    const StepInputs s = load_step_inputs(smp, n_u, chunk_lv, fallback_t, lds_i, blockIdx.x);
    const M3<F> ex = block_exclusive_product<F>(step_of<F>(s), lds_m);
    const int i = blockIdx.x * kChunk + threadIdx.x;
    if (i >= n_u) return;
    V3<double> C3 = mk(0.0, 0.0, 0.0);
    if (frenet) {
        V3<double> o[4];
        sample_derivs_any<3>(path, i, n_u, o);
        C3 = o[3];
    }
    const LawSample lw = law_at(has_law ? &law : nullptr, i, n_u, du_scale);
    write_row_ext<F, T>(s, ex, r_in + 3 * (size_t)blockIdx.x, smp_get(smp, nu, 1, i), smp_get(smp, nu, 2, i), C3,
                        frenet, lw, reorth, rows + kRowExt * (size_t)i);
}

// ------------------------------------------------------------- launchers

int frame_chunk_size() { return kChunk; }

template <class F, class T>
hipError_t launch_prep(const DCurve& path, int n_u, const DCurve& prof, int n_v, double* smp, int* chunk_lv,
                       int* chunk_fix, double* fallback_t, F* agg, T* ptab, hipStream_t st)
{
    const int ncu = (n_u + kChunk - 1) / kChunk;
    const int ncv = (n_v + kBlock - 1) / kBlock;
    const dim3 grid(ncu + ncv);
#define SWEEP_CASE(P) \
    case P: hipLaunchKernelGGL((k_prep<P, F, T>), grid, dim3(kBlock), 0, st, path, n_u, prof, n_v, ncu, smp, \
                               chunk_lv, chunk_fix, fallback_t, agg, ptab); break;
    switch (path.p) {
        SWEEP_CASE(1) SWEEP_CASE(2) SWEEP_CASE(3) SWEEP_CASE(4) SWEEP_CASE(5) SWEEP_CASE(6) SWEEP_CASE(7)
    default: return hipErrorInvalidValue;
    }
#undef SWEEP_CASE
    return hipGetLastError();
}

template <class F, class T>
hipError_t launch_frame(const double* smp, int n_u, const int* chunk_lv, const int* chunk_fix,
                        const double* fallback_t, InitialNormal n0, int reorth, F* agg, F* r_in, T* rows,
                        hipStream_t st, const FrameExt* ext)
{
    const int nc = (n_u + kChunk - 1) / kChunk;
    if (!ext && nc <= kBlock) {
        hipLaunchKernelGGL((k_frame_apply_fused<F, T>), dim3(nc), dim3(kBlock), 0, st, smp, n_u, chunk_lv, chunk_fix,
                           fallback_t, agg, n0, reorth, rows);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_frame_carry<F>, dim3(1), dim3(kBlock), 0, st, agg, nc, smp, n_u, chunk_lv, chunk_fix,
                       fallback_t, n0, r_in);
    if (ext)
        hipLaunchKernelGGL((k_frame_apply_ext<F, T>), dim3(nc), dim3(kBlock), 0, st, smp, n_u, chunk_lv, fallback_t,
                           r_in, reorth, ext->path, ext->frenet, ext->law, ext->has_law, ext->du_scale, rows);
    else
        hipLaunchKernelGGL((k_frame_apply<F, T>), dim3(nc), dim3(kBlock), 0, st, smp, n_u, chunk_lv, fallback_t,
                           r_in, reorth, rows);
    return hipGetLastError();
}
#define SWEEP_INST(F, T)                                                                                          \
    template hipError_t launch_prep<F, T>(const DCurve&, int, const DCurve&, int, double*, int*, int*, double*, F*, \
                                          T*, hipStream_t);                                                        \
    template hipError_t launch_frame<F, T>(const double*, int, const int*, const int*, const double*, InitialNormal, \
                                           int, F*, F*, T*, hipStream_t, const FrameExt*);
SWEEP_INST(double, float)
SWEEP_INST(double, double)
SWEEP_INST(float, float)
SWEEP_INST(float, double)
#undef SWEEP_INST

}  // namespace sweep
