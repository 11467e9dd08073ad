// frame_kernels.hip -- the rotation-minimizing frame of a single sweep as a
// parallel prefix product of 3x3 rotations over runs of K consecutive
// u-samples per thread (frame_walk.hpp), in two or three launches:
//
// k_prep          per chunk of kBlock*K samples: every run's product of step
//                 rotations and resolved first tangent (a per-run record),
//                 the chunk's product A_c, its last sample with C' != 0 and
//                 that sample's tangent.  A chunk whose first sample has
//                 C' = 0 needs the tangent of an earlier chunk: it is flagged
//                 and its records are formed later.  Extra blocks write the
//                 profile table (S, S' in the output precision).
// k_frame_carry   one block, more than kBlock chunks (or a frame mode or
//                 law): records and products of the flagged chunks, then the
//                 scan of the A_c giving the normal entering each chunk,
//                 r_in[c] = (A_{c-1} ... A_0) r_0.  (A separate launch: a
//                 last-block hand-off inside k_prep would need a device-scope
//                 fence per block, whose L2 write-back across the eight XCDs
//                 costs more than the launch.)
// k_frame_apply   per chunk: block exclusive product of the run products
//                 applied to r_in[c], then each thread walks its run writing
//                 row records (x, r, s, t, |C'|, a, b) in the output
//                 precision, re-orthonormalised if asked.
// k_frame_apply_fused  up to kBlock*kFusedGroup chunks (no frame mode or law): replaces
//                 k_frame_carry + k_frame_apply; block b forms its entry
//                 normal as the ordered block product of the chunk products
//                 below it (flagged chunks' products formed in the block),
//                 applied to r_0.
#include "frame_walk.hpp"

namespace sweep {

// Runs per chunk (one per thread) and the run length K for n_u samples:
// the smallest power of two up to 16 that keeps the chunks at most
// kBlock*kFusedGroup (the fused route): about 131,072 threads or more, two
// waves per SIMD on 256 CUs, which the walk's register use allows.
int frame_run_length(int n_u)
{
    int K = 1;
    while (K < 16 && (long long)kBlock * kBlock * kFusedGroup * K < (long long)n_u) K *= 2;
    return K;
}
int frame_chunks(int n_u)
{
    const long long cs = (long long)kBlock * frame_run_length(n_u);
    return (int)(((long long)n_u + cs - 1) / cs);
}

template <class F>
__device__ __forceinline__ void store_record(double* __restrict__ q, const M3<F>& A, V3<double> t_first)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) q[e] = (double)A.m[e];
    q[9] = t_first.x; q[10] = t_first.y; q[11] = t_first.z;
}
template <class F>
__device__ __forceinline__ void load_record(const double* __restrict__ q, M3<F>& A, V3<double>& t_first)
{
#pragma unroll
    for (int e = 0; e < 9; ++e) A.m[e] = (F)q[e];
    t_first = mk(q[9], q[10], q[11]);
}

// Resolved tangent of sample 0 (the first run's record: chunk 0 is never flagged).
__device__ __forceinline__ V3<double> first_tangent(const double* __restrict__ trec)
{
    return mk(trec[9], trec[10], trec[11]);
}

// Blocks [0, ncu): run records and chunk products; blocks [ncu, ncu + ncv):
// profile table.
template <int P, class F, class T>
__global__ __launch_bounds__(kBlock) void k_prep(DCurve path, int n_u, int K, DCurve prof, int n_v, int ncu,
                                                 double* __restrict__ trec, int* __restrict__ chunk_lv,
                                                 double* __restrict__ chunk_tl, int* __restrict__ chunk_fix,
                                                 double* __restrict__ fallback_t, F* __restrict__ agg,
                                                 T* __restrict__ ptab)
{
    if ((int)blockIdx.x >= ncu) {
        const int j = ((int)blockIdx.x - ncu) * kBlock + threadIdx.x;
        if (j < n_v) write_profile<T>(prof, j, n_v, ptab);
        return;
    }
    __shared__ ChunkWalkLds L;
    __shared__ M3<F> lds_m[kWaves];
    const int c = blockIdx.x;
    const int base = c * kBlock * K;
    const V3<double> fb = first_leg(path);
    if (c == 0 && threadIdx.x == 0) {
        // used only when C'(u_0) = 0
        fallback_t[0] = fb.x; fallback_t[1] = fb.y; fallback_t[2] = fb.z;
    }
    RunInfo<P, F> R;
    int clv;
    V3<double> ctl;
    const bool ok = chunk_products<P, F>(path, n_u, base, K, c == 0, fb, L, R, clv, ctl);
    if (threadIdx.x == 0) {
        chunk_lv[c] = clv;
        chunk_tl[3 * c] = ctl.x; chunk_tl[3 * c + 1] = ctl.y; chunk_tl[3 * c + 2] = ctl.z;
        chunk_fix[c] = ok ? 0 : 1;
    }
    if (!ok) return;   // block-uniform: records formed by the carry or the fused apply
    store_record<F>(trec + kRunRec * ((size_t)c * kBlock + threadIdx.x), R.A, R.t_first);
    const M3<F> prod = block_product<F>(R.A, lds_m);
    if (threadIdx.x < 9) agg[9 * (size_t)c + threadIdx.x] = prod.m[threadIdx.x];
}

// Tangent carried into a chunk whose entry is the last sample with C' != 0
// below it (index lv, -1 if none): that sample's chunk's recorded tangent.
__device__ __forceinline__ V3<double> entry_tangent(int lv, int chunk_samples, const double* __restrict__ chunk_tl,
                                                    V3<double> fb)
{
    if (lv < 0) return fb;
    const int o = lv / chunk_samples;
    return mk(chunk_tl[3 * o], chunk_tl[3 * o + 1], chunk_tl[3 * o + 2]);
}

// One block: records and products of the flagged chunks, then
// r_in[c] = (A_{c-1} ... A_0) r_0 for every chunk.
template <int P, class F>
__global__ __launch_bounds__(kBlock) void k_frame_carry(DCurve path, int n_u, int K, F* __restrict__ agg,
                                                        int n_chunks, const int* __restrict__ chunk_lv,
                                                        const double* __restrict__ chunk_tl,
                                                        const int* __restrict__ chunk_fix,
                                                        const double* __restrict__ fallback_t,
                                                        double* __restrict__ trec, InitialNormal n0,
                                                        F* __restrict__ r_in)
{
    __shared__ ChunkWalkLds L;
    __shared__ M3<F> lds_m[kWaves];
    __shared__ int lx[kBlock];
    __shared__ int lf[kBlock];
    const int cs = kBlock * K;
    const V3<double> fb = mk(fallback_t[0], fallback_t[1], fallback_t[2]);
    int below = -1;   // last sample with C' != 0 in the chunks before this range
    for (int base = 0; base < n_chunks; base += kBlock) {
        const int c = base + threadIdx.x;
        const int lv = c < n_chunks ? chunk_lv[c] : -1;
        const int fl = c < n_chunks ? chunk_fix[c] : 0;
        int tot, last_flagged;
        const int x = block_exclusive_max(lv, L.ii, tot);
        lx[threadIdx.x] = max(x, below);
        lf[threadIdx.x] = fl;
        block_exclusive_max(fl ? (int)threadIdx.x : -1, L.ii, last_flagged);   // also orders lx, lf
        for (int f = 0; f <= last_flagged; ++f) {   // uniform; skipped when none
            if (!lf[f]) continue;
            const int cf = base + f;
            RunInfo<P, F> R;
            int clv;
            V3<double> ctl;
            chunk_products<P, F>(path, n_u, cf * cs, K, true, entry_tangent(lx[f], cs, chunk_tl, fb), L, R, clv, ctl);
            store_record<F>(trec + kRunRec * ((size_t)cf * kBlock + threadIdx.x), R.A, R.t_first);
            const M3<F> prod = block_product<F>(R.A, lds_m);
            if (threadIdx.x < 9) agg[9 * (size_t)cf + threadIdx.x] = prod.m[threadIdx.x];
            __threadfence_block();
            __syncthreads();
        }
        below = max(below, tot);
    }
    carry_scan<F>(agg, n_chunks, initial_normal(first_tangent(trec), n0), r_in, lds_m);
}

template <int P, class F, class T, bool EXT>
__global__ __launch_bounds__(kBlock) void k_frame_apply(DCurve path, int n_u, int K, const double* __restrict__ trec,
                                                        const F* __restrict__ r_in, int reorth, T* __restrict__ rows,
                                                        int frenet, DCurve law, int has_law, double du_scale)
{
    __shared__ M3<F> lds_m[kWaves];
    const int c = blockIdx.x;
    M3<F> A;
    V3<double> t_first;
    load_record<F>(trec + kRunRec * ((size_t)c * kBlock + threadIdx.x), A, t_first);
    const M3<F> ex = block_exclusive_product<F>(A, lds_m);
    const V3<F> r = apply(ex, mk(r_in[3 * c], r_in[3 * c + 1], r_in[3 * c + 2]));
    const int i0 = c * kBlock * K + threadIdx.x * K;
    if (EXT)
        run_rows<P, 3, F>(path, n_u, i0, K, t_first, r, ExtRows<F, T>{rows, reorth, frenet, has_law, n_u, law, du_scale});
    else
        run_rows<P, 2, F>(path, n_u, i0, K, t_first, r, PlainRows<F, T>{rows, reorth});
}

// k_frame_apply without k_frame_carry, for at most kBlock*G chunks: thread c
// holds the ordered product A_c of chunks [cG, cG + G) below b (identity
// above); the products of flagged chunks (not formed by k_prep) are formed
// here, as k_frame_carry does, in increasing order, and the owning thread
// multiplies them in at their place.  The ordered block product of the A_c
// applied to r_0 is the block's entry normal.  A flagged chunk b also forms
// its own run records here.
template <int P, class F, class T>
__global__ __launch_bounds__(kBlock) void k_frame_apply_fused(DCurve path, int n_u, int K, int G,
                                                              const double* __restrict__ trec,
                                                              const int* __restrict__ chunk_lv,
                                                              const double* __restrict__ chunk_tl,
                                                              const int* __restrict__ chunk_fix,
                                                              const double* __restrict__ fallback_t,
                                                              const F* __restrict__ agg, InitialNormal n0, int reorth,
                                                              T* __restrict__ rows)
{
    __shared__ ChunkWalkLds L;
    __shared__ M3<F> lds_m[kWaves];
    __shared__ M3<F> lds_fix;
    __shared__ int lflag[kBlock];
    __shared__ int lx[kBlock];
    __shared__ F lds_r[3];
    const int b = blockIdx.x, c = threadIdx.x;
    const int cs = kBlock * K;
    const int g0 = c * G, g1 = min(g0 + G, b);   // this thread's chunks below b: [g0, g1)
    const V3<double> fb = mk(fallback_t[0], fallback_t[1], fallback_t[2]);
    int flagged = 0, lv = -1;
    for (int cc = g0; cc < g1; ++cc) {
        flagged |= chunk_fix[cc];
        lv = max(lv, chunk_lv[cc]);
    }
    int lv_below_b, last_flagged;
    lx[c] = block_exclusive_max(lv, L.ii, lv_below_b);   // last valid sample below chunk g0
    lflag[c] = flagged;
    block_exclusive_max(flagged ? c : -1, L.ii, last_flagged);   // also orders lx, lflag
    M3<F> A = ident<F>();
    int next = g0;   // the first chunk of the group not yet in A
    for (int t = 0; t <= last_flagged; ++t) {   // uniform; skipped when none
        if (!lflag[t]) continue;
        int lvf = lx[t];
        for (int f = t * G; f < min(t * G + G, b); ++f) {
            if (chunk_fix[f]) {
                RunInfo<P, F> R;
                int clv;
                V3<double> ctl;
                chunk_products<P, F>(path, n_u, f * cs, K, true, entry_tangent(lvf, cs, chunk_tl, fb), L, R, clv,
                                     ctl);
                const M3<F> prod = block_product<F>(R.A, lds_m);
                if (threadIdx.x == 0) lds_fix = prod;
                __syncthreads();
                if (c == t) {
                    for (; next < f; ++next) {
                        M3<F> M;
#pragma unroll
                        for (int e = 0; e < 9; ++e) M.m[e] = agg[9 * (size_t)next + e];
                        A = mul(M, A);
                    }
                    A = mul(lds_fix, A);
                    next = f + 1;
                }
                __syncthreads();
            }
            lvf = max(lvf, chunk_lv[f]);
        }
    }
    for (; next < g1; ++next) {
        M3<F> M;
#pragma unroll
        for (int e = 0; e < 9; ++e) M.m[e] = agg[9 * (size_t)next + e];
        A = mul(M, A);
    }
    const M3<F> Pb = block_product<F>(A, lds_m);   // A_{b-1} ... A_0, valid in wave 0
    if (threadIdx.x == 0) {
        const V3<F> r = apply(Pb, cvt<F>(initial_normal(first_tangent(trec), n0)));
        lds_r[0] = r.x; lds_r[1] = r.y; lds_r[2] = r.z;
    }
    __syncthreads();
    const V3<F> rin = mk(lds_r[0], lds_r[1], lds_r[2]);
    // this chunk's run records
    RunInfo<P, F> R;
    V3<double> t_first;
    M3<F> Ar;
    if (chunk_fix[b]) {   // block-uniform
        int clv;
        V3<double> ctl;
        chunk_products<P, F>(path, n_u, b * cs, K, true, entry_tangent(lv_below_b, cs, chunk_tl, fb), L, R, clv, ctl);
        Ar = R.A;
        t_first = R.t_first;
    } else {
        load_record<F>(trec + kRunRec * ((size_t)b * kBlock + threadIdx.x), Ar, t_first);
    }
    const M3<F> ex = block_exclusive_product<F>(Ar, lds_m);
    const int i0 = b * cs + threadIdx.x * K;
    run_rows<P, 2, F>(path, n_u, i0, K, t_first, apply(ex, rin), PlainRows<F, T>{rows, reorth});
}

// ------------------------------------------------------------- launchers

template <class F, class T>
hipError_t launch_prep(const DCurve& path, int n_u, const DCurve& prof, int n_v, const FrameWork& w, T* ptab,
                       hipStream_t st)
{
    const int K = frame_run_length(n_u);
    const int ncu = frame_chunks(n_u);
    const int ncv = (n_v + kBlock - 1) / kBlock;
#define SWEEP_CASE(P) \
    case P: hipLaunchKernelGGL((k_prep<P, F, T>), dim3(ncu + ncv), dim3(kBlock), 0, st, path, n_u, K, prof, n_v, \
                               ncu, w.trec, w.chunk_lv, w.chunk_tl, w.chunk_fix, w.fallback_t, (F*)w.agg, ptab); break;
    switch (path.p) {
        SWEEP_CASE(1) SWEEP_CASE(2) SWEEP_CASE(3) SWEEP_CASE(4) SWEEP_CASE(5) SWEEP_CASE(6) SWEEP_CASE(7)
    default: return hipErrorInvalidValue;
    }
#undef SWEEP_CASE
    return hipGetLastError();
}

template <int P, class F, class T>
static void launch_frame_p(const DCurve& path, int n_u, const FrameWork& w, InitialNormal n0, int reorth, T* rows,
                           hipStream_t st, const FrameExt* ext)
{
    const int K = frame_run_length(n_u);
    const int nc = frame_chunks(n_u);
    if (!ext && nc <= kBlock * kFusedGroup) {
        const int G = (nc + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((k_frame_apply_fused<P, F, T>), dim3(nc), dim3(kBlock), 0, st, path, n_u, K, G, w.trec,
                           w.chunk_lv, w.chunk_tl, w.chunk_fix, w.fallback_t, (const F*)w.agg, n0, reorth, rows);
        return;
    }
    hipLaunchKernelGGL((k_frame_carry<P, F>), dim3(1), dim3(kBlock), 0, st, path, n_u, K, (F*)w.agg, nc, w.chunk_lv,
                       w.chunk_tl, w.chunk_fix, w.fallback_t, w.trec, n0, (F*)w.r_in);
    if (ext)
        hipLaunchKernelGGL((k_frame_apply<P, F, T, true>), dim3(nc), dim3(kBlock), 0, st, path, n_u, K, w.trec,
                           (const F*)w.r_in, reorth, rows, ext->frenet, ext->law, ext->has_law, ext->du_scale);
    else
        hipLaunchKernelGGL((k_frame_apply<P, F, T, false>), dim3(nc), dim3(kBlock), 0, st, path, n_u, K, w.trec,
                           (const F*)w.r_in, reorth, rows, 0, path, 0, 0.0);
}

template <class F, class T>
hipError_t launch_frame(const DCurve& path, int n_u, const FrameWork& w, InitialNormal n0, int reorth, T* rows,
                        hipStream_t st, const FrameExt* ext)
{
    switch (path.p) {
    case 1: launch_frame_p<1, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 2: launch_frame_p<2, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 3: launch_frame_p<3, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 4: launch_frame_p<4, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 5: launch_frame_p<5, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 6: launch_frame_p<6, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    case 7: launch_frame_p<7, F, T>(path, n_u, w, n0, reorth, rows, st, ext); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define SWEEP_INST(F, T)                                                                                        \
    template hipError_t launch_prep<F, T>(const DCurve&, int, const DCurve&, int, const FrameWork&, T*,          \
                                          hipStream_t);                                                          \
    template hipError_t launch_frame<F, T>(const DCurve&, int, const FrameWork&, InitialNormal, int, T*,         \
                                           hipStream_t, const FrameExt*);
SWEEP_INST(double, float)
SWEEP_INST(double, double)
SWEEP_INST(float, float)
SWEEP_INST(float, double)
#undef SWEEP_INST

}  // namespace sweep
