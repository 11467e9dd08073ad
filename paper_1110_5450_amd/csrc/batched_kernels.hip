// batched_kernels.hip -- a batch of independent sweeps, replayed as one HIP
// graph:
//
// kb_profile  one block per (sweep, chunk of 256 v-samples): profile tables.
// kb_frame    one block per sweep, one launch per path degree present (the
//             degree is a template parameter, so the B-spline arrays stay in
//             registers); sweeps are listed longest first.  Each thread walks
//             a run of K consecutive u-samples (K = 1 .. 16, so that a sweep
//             of up to 4096 samples is one chunk of kBlock runs): the run
//             products, the block's exclusive product scan, then the row
//             records (frame_walk.hpp).  Longer sweeps walk their chunks in
//             order, carrying the entering normal and the last resolved
//             tangent in registers: no cross-block carry is needed.
// kb_frame_wave  one wave per sweep of at most kWaveMaxU u-samples.
// kb_surface  one block per tile of 256*K (K = 1, 2, 4, 8) consecutive
//             vertices of one sweep, rows staged in LDS, one vertex per lane
//             per step, six plane stores.
// kb_arc_*    arc-length (or curvature-adaptive) u-samples of every path:
//             piece lengths, one cumulative table per sweep, sample
//             parameters (arclength.hpp, as for a single sweep).
//
// The frame steps are the single-sweep kernels' device functions; the
// batch groups a sweep's step rotations into runs differently, so a batched
// sweep and the same sweep alone agree to rounding.
#include "arclength.hpp"
#include "frame_walk.hpp"
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

// Arc-length tables of the batch's paths, one launch per path degree P (RAT:
// the paths carry weights).  Pieces: a block per kWaves spans of one sweep
// (chunk = (sweep, first span index)), a wave per span.
template <int P, bool ADAPT, bool RAT>
__global__ __launch_bounds__(kBlock) void kb_arc_pieces(const BatchDesc* __restrict__ descs,
                                                        const int2* __restrict__ chunks,
                                                        const double* __restrict__ path_ctrl,
                                                        const double* __restrict__ path_w,
                                                        const double* __restrict__ knots, double lam,
                                                        double* __restrict__ len)
{
    __shared__ double setup[kWaves][SpanDeriv<P>::kDoubles];
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const int w = threadIdx.x >> 6, si = ch.y + w;
    if (d.p_path != P || si >= d.n_path - P) return;   // whole waves (the list holds degree-P sweeps only)
    arc_span<P, ADAPT, RAT>(path_of(d, path_ctrl, path_w, knots), si, threadIdx.x & 63, lam, setup[w],
                            len + d.arc_off);
}

// One block per sweep: its cumulative table at arc_off + k (one entry more
// than its pieces).
__global__ __launch_bounds__(kScanThreads) void kb_arc_cumsum(const BatchDesc* __restrict__ descs,
                                                              const double* __restrict__ len,
                                                              double* __restrict__ cum)
{
    const BatchDesc d = descs[blockIdx.x];
    arc_cumsum_block(len + d.arc_off, arc_piece_count(d.n_path, d.p_path), cum + d.arc_off + blockIdx.x);
}

// Sample parameters (one launch per path degree): a block per 32 u-samples
// of one sweep (chunk = (sweep, first sample)), kArcLanes lanes per sample;
// parameters and spans at the sweep's row offset.
template <int P, bool ADAPT, bool RAT>
__global__ __launch_bounds__(kBlock) void kb_arc_params(const BatchDesc* __restrict__ descs,
                                                        const int2* __restrict__ chunks,
                                                        const double* __restrict__ path_ctrl,
                                                        const double* __restrict__ path_w,
                                                        const double* __restrict__ knots, double lam,
                                                        const double* __restrict__ cum, double* __restrict__ su,
                                                        int* __restrict__ ss)
{
    __shared__ double coarse[kArcCoarseMax];
    __shared__ double setup[kBlock / kArcLanes][SpanDeriv<P>::kDoubles];
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    if (d.p_path != P) return;   // the list holds degree-P sweeps only
    const int npc = arc_piece_count(d.n_path, d.p_path), cs = arc_coarse_stride(npc);
    const int nc = npc / cs + 1;
    const double* cumk = cum + d.arc_off + ch.x;
    for (int k = threadIdx.x; k < nc; k += kBlock) coarse[k] = cumk[(long long)k * cs];
    __syncthreads();
    const int i = ch.y + (int)(threadIdx.x / kArcLanes);
    if (i >= d.n_u) return;   // whole lane groups
    arc_param<P, ADAPT, RAT>(path_of(d, path_ctrl, path_w, knots), i, threadIdx.x & (kArcLanes - 1), d.n_u, npc, cs,
                             nc, lam, cumk, coarse, setup[threadIdx.x / kArcLanes], su + d.row_off,
                             ss + d.row_off);
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

// Run length of a batched sweep: the smallest power of two up to
// kMaxRun with kBlock*K >= n_u (a sweep of up to kBlock*kMaxRun u-samples is
// one chunk).
__device__ __forceinline__ int batch_run_length(int n_u)
{
    int K = 1;
    while (K < kMaxRun && kBlock * K < n_u) K *= 2;
    return K;
}

// Pass 2 of a run in a batched frame kernel: plain row records (16 values),
// or with EXT the extended records of the batch's frame mode and law (ND = 3:
// the Frenet frame uses the third derivative; the law's dl/du is fx.law_len
// over this path's domain length).
template <int P, class F, class T, bool EXT, class C>
__device__ __forceinline__ void walk_rows(const C& path, const DCurve& gpath, const BatchDesc& d, int n_u, int i0,
                                          int K, V3<double> t_first, V3<F> r, int reorth, const BatchFrameExt& fx,
                                          T* __restrict__ rows)
{
    if constexpr (EXT) {
        const double du = fx.has_law ? fx.law_len / (knot(gpath, gpath.n) - knot(gpath, gpath.p)) : 0.0;
        run_rows<P, 3, F>(path, n_u, i0, K, t_first, r,
                          ExtRows<F, T>{rows + kRowExt * (size_t)d.row_off, reorth, fx.frenet, fx.has_law, n_u, fx.law,
                                        du});
    } else {
        run_rows<P, 2, F>(path, n_u, i0, K, t_first, r, PlainRows<F, T>{rows + 16 * (size_t)d.row_off, reorth});
    }
}

// Row records of a sweep of at most kBlock*kMaxRun u-samples whose path has
// degree P: one block per sweep, one chunk.  The path is staged in LDS
// (knots, control points, weights, per-span reciprocals; kLdsPathDoubles of
// dynamic LDS): knot span changes read LDS only.
template <int P, class F, class T, bool EXT, bool ARC>
__global__ __launch_bounds__(kBlock) void kb_frame(const BatchDesc* __restrict__ descs,
                                                   const int* __restrict__ sweeps,
                                                   const double* __restrict__ path_ctrl,
                                                   const double* __restrict__ path_w,
                                                   const double* __restrict__ knots, InitialNormal n0, int reorth,
                                                   T* __restrict__ rows, BatchFrameExt fx)
{
    __shared__ ChunkWalkLds L;
    __shared__ M3<F> lds_m[kWaves];
    __shared__ double lt0[3];
    extern __shared__ double lds_path[];   // kLdsPathDoubles
    const BatchDesc d = descs[sweeps[blockIdx.x]];
    DCurve gpath = path_of(d, path_ctrl, path_w, knots);
    LdsCurve path = stage_path<P>(gpath, lds_path);
    if constexpr (ARC) {   // arc-length samples: parameters and spans from the sweep's tables
        gpath.su = path.su = fx.su + d.row_off;
        gpath.ss = path.ss = fx.ss + d.row_off;
    }
    const int n_u = d.n_u;
    const int K = batch_run_length(n_u);
    RunInfo<P, F> R;
    int clv;
    V3<double> ctl;
    chunk_products<P, F>(path, n_u, 0, K, true, first_leg(gpath), L, R, clv, ctl);
    // r_0 from the resolved t_0 (sample 0 is thread 0's)
    if (threadIdx.x == 0) { lt0[0] = R.t_first.x; lt0[1] = R.t_first.y; lt0[2] = R.t_first.z; }
    __syncthreads();
    const V3<F> rin = cvt<F>(initial_normal(mk(lt0[0], lt0[1], lt0[2]), n0));
    const M3<F> ex = block_exclusive_product<F>(R.A, lds_m);
    walk_rows<P, F, T, EXT>(path, gpath, d, n_u, (int)threadIdx.x * K, K, R.t_first, apply(ex, rin), reorth, fx, rows);
}

// Run length of a sweep framed by one wave: the smallest power of two up to
// kMaxRun with 64*K >= n_u (at most 4 for kWaveMaxU = 256).
__device__ __forceinline__ int wave_run_length(int n_u)
{
    int K = 1;
    while (K < kMaxRun && 64 * K < n_u) K *= 2;
    return K;
}

// Row records of sweeps of at most kWaveMaxU u-samples, one wave per sweep
// (four sweeps per block, no block barriers): lane l owns the run of K
// samples from l*K.  The tangent carries and the exclusive product of the
// run products are wave scans (cross-lane moves); the path is read from
// global memory.  Entries of -1 in the sweep list (padding to whole blocks)
// are skipped.
template <int P, class F, class T, bool EXT, bool ARC>
__global__ __launch_bounds__(kBlock) void kb_frame_wave(const BatchDesc* __restrict__ descs,
                                                        const int* __restrict__ sweeps,
                                                        const double* __restrict__ path_ctrl,
                                                        const double* __restrict__ path_w,
                                                        const double* __restrict__ knots, InitialNormal n0,
                                                        int reorth, T* __restrict__ rows, BatchFrameExt fx)
{
    const int lane = threadIdx.x & 63;
    const int k = sweeps[blockIdx.x * kWaves + (threadIdx.x >> 6)];
    if (k < 0) return;   // wave-uniform
    const BatchDesc d = descs[k];
    DCurve path = path_of(d, path_ctrl, path_w, knots);
    if constexpr (ARC) {   // arc-length samples
        path.su = fx.su + d.row_off;
        path.ss = fx.ss + d.row_off;
    }
    const int n_u = d.n_u;
    const int K = wave_run_length(n_u);
    const int i0 = lane * K;
    const V3<double> t_entry = first_leg(path);
    RunInfo<P, F> R = run_product<P, F>(path, n_u, i0, K, t_entry);
    // last sample with C' != 0 below this lane's run, and its tangent
    int src = R.last_valid;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        const int o = __shfl_up(src, dd, 64);
        if (lane >= dd) src = max(src, o);
    }
    src = __shfl_up(src, 1, 64);
    if (lane == 0) src = -1;
    const int owner = src >= 0 ? src / K : 0;
    V3<double> tc = mk(__shfl(R.t_last_valid.x, owner, 64), __shfl(R.t_last_valid.y, owner, 64),
                       __shfl(R.t_last_valid.z, owner, 64));
    if (src < 0) tc = t_entry;
    // runs whose first sample has C' = 0 walk again with the carry resolved
    // (lane 0's carry is the known entry: it never needs to)
    if (i0 < n_u && !R.first_valid && lane > 0) R = run_product<P, F>(path, n_u, i0, K, tc);
    // r_0 from the resolved t_0 (lane 0's first sample)
    const V3<double> t0 = mk(__shfl(R.t_first.x, 0, 64), __shfl(R.t_first.y, 0, 64), __shfl(R.t_first.z, 0, 64));
    const V3<F> rin = cvt<F>(initial_normal(t0, n0));
    const M3<F> ex = wave_shift_up1<F>(wave_inclusive_product<F>(R.A));
    walk_rows<P, F, T, EXT>(path, path, d, n_u, i0, K, R.t_first, apply(ex, rin), reorth, fx, rows);
}

// The same for longer sweeps: the block walks chunks of kBlock*kMaxRun
// samples in order, carrying the entering normal and the last resolved
// tangent.  (A kernel of its own: the loop's carried state raises the
// register allocation above that of the one-chunk kernel.)
template <int P, class F, class T, bool EXT, bool ARC>
__global__ __launch_bounds__(kBlock) void kb_frame_long(const BatchDesc* __restrict__ descs,
                                                        const int* __restrict__ sweeps,
                                                        const double* __restrict__ path_ctrl,
                                                        const double* __restrict__ path_w,
                                                        const double* __restrict__ knots, InitialNormal n0,
                                                        int reorth, T* __restrict__ rows, BatchFrameExt fx)
{
    __shared__ ChunkWalkLds L;
    __shared__ M3<F> lds_m[kWaves];
    __shared__ double lt0[3];
    const BatchDesc d = descs[sweeps[blockIdx.x]];
    DCurve path = path_of(d, path_ctrl, path_w, knots);
    if constexpr (ARC) {   // arc-length samples
        path.su = fx.su + d.row_off;
        path.ss = fx.ss + d.row_off;
    }
    const int n_u = d.n_u;
    const int K = batch_run_length(n_u);
    const int cs = kBlock * K;
    V3<double> t_entry = first_leg(path);
    V3<F> rin = mk(F(0), F(0), F(0));
    for (int base = 0; base < n_u; base += cs) {
        RunInfo<P, F> R;
        int clv;
        V3<double> ctl;
        chunk_products<P, F>(path, n_u, base, K, true, t_entry, L, R, clv, ctl);
        if (base == 0) {
            if (threadIdx.x == 0) { lt0[0] = R.t_first.x; lt0[1] = R.t_first.y; lt0[2] = R.t_first.z; }
            __syncthreads();
            rin = cvt<F>(initial_normal(mk(lt0[0], lt0[1], lt0[2]), n0));
        }
        M3<F> total;
        const M3<F> ex = block_exclusive_product<F>(R.A, lds_m, total);
        walk_rows<P, F, T, EXT>(path, path, d, n_u, base + (int)threadIdx.x * K, K, R.t_first, apply(ex, rin), reorth,
                                fx, rows);
        rin = apply(total, rin);
        t_entry = ctl;   // the last resolved tangent up to this chunk's end
    }
}

// K = vertices per lane (tile of 256*K vertices per block).
template <class T, bool NRM, bool NT, int K, int RL>
__global__ __launch_bounds__(kBlock) void kb_surface(const BatchDesc* __restrict__ descs,
                                                     const int2* __restrict__ tiles, const T* __restrict__ rows,
                                                     const T* __restrict__ ptab, T* __restrict__ pos,
                                                     T* __restrict__ nrm)
{
    __shared__ T lrow[kMaxLdsRows * RL];
    const int2 tl = tiles[blockIdx.x];
    const BatchDesc d = descs[tl.x];
    const FastDiv dv{d.fd_m, d.fd_shift, d.n_v};
    const long long N = (long long)d.n_u * (long long)d.n_v;
    const long long v0 = tl.y;
    const long long vlast = min(N, v0 + kBlock * K) - 1;
    const T* rows_k = rows + RL * d.row_off;
    const int ilo = fdiv((unsigned)v0, dv);
    const int nrow = fdiv((unsigned)vlast, dv) - ilo + 1;
    const bool staged = nrow <= kMaxLdsRows;
    if (staged)
        for (int e = threadIdx.x; e < nrow * RL; e += kBlock) lrow[e] = rows_k[RL * (size_t)ilo + e];
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
                vertex_rl<RL, T>(base + RL * (size_t)(vi[k] - row0), qv[k][0], qv[k][1], qv[k][2], qv[k][3],
                                 qv[k][4], qv[k][5], X[k], Nn[k]);
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

template <class T, bool NRM, bool NT, int RL>
static const void* surface_for(int K)
{
    switch (K) {
    case 1: return (const void*)&kb_surface<T, NRM, NT, 1, RL>;
    case 2: return (const void*)&kb_surface<T, NRM, NT, 2, RL>;
    case 4: return (const void*)&kb_surface<T, NRM, NT, 4, RL>;
    default: return (const void*)&kb_surface<T, NRM, NT, 8, RL>;
    }
}

template <class T, int RL>
static const void* surface_pick(bool nrm, bool nt, int K)
{
    if (nrm) return nt ? surface_for<T, true, true, RL>(K) : surface_for<T, true, false, RL>(K);
    return nt ? surface_for<T, false, true, RL>(K) : surface_for<T, false, false, RL>(K);
}

// Frame kernels of a frame precision, output precision, record kind and
// sampling (ARC: the sweeps' sample parameters and spans come from the
// arc-length tables).
template <class F, class T, bool EXT, bool ARC>
static void pick_frames(BatchedKernels& k)
{
    k.frame[0] = k.frame_long[0] = k.frame_wave[0] = nullptr;
#define SWEEP_DEG(P)                                                                  \
    k.frame[P] = (const void*)&kb_frame<P, F, T, EXT, ARC>;                          \
    k.frame_long[P] = (const void*)&kb_frame_long<P, F, T, EXT, ARC>;                \
    k.frame_wave[P] = (const void*)&kb_frame_wave<P, F, T, EXT, ARC>;
    SWEEP_DEG(1) SWEEP_DEG(2) SWEEP_DEG(3) SWEEP_DEG(4) SWEEP_DEG(5) SWEEP_DEG(6) SWEEP_DEG(7)
#undef SWEEP_DEG
}

template <bool ADAPT, bool RAT>
static void pick_arc(BatchedKernels& k)
{
    k.arc_pieces[0] = k.arc_params[0] = nullptr;
#define SWEEP_DEG(P)                                                   \
    k.arc_pieces[P] = (const void*)&kb_arc_pieces<P, ADAPT, RAT>;     \
    k.arc_params[P] = (const void*)&kb_arc_params<P, ADAPT, RAT>;
    SWEEP_DEG(1) SWEEP_DEG(2) SWEEP_DEG(3) SWEEP_DEG(4) SWEEP_DEG(5) SWEEP_DEG(6) SWEEP_DEG(7)
#undef SWEEP_DEG
    k.arc_cumsum = (const void*)&kb_arc_cumsum;
}

// Extended records (a frame mode or a law) and arc-length sampling with the
// FP64 frame only, not together: the caller rejects the other combinations.
template <class F, class T>
static BatchedKernels pick(bool nrm, bool nt, int K, bool ext, bool arc, bool adaptive, bool rat)
{
    BatchedKernels k;
    k.profile = (const void*)&kb_profile<T>;
    if constexpr (sizeof(F) == 8) {
        if (ext) pick_frames<F, T, true, false>(k);
        else if (arc) pick_frames<F, T, false, true>(k);
        else pick_frames<F, T, false, false>(k);
    } else {
        pick_frames<F, T, false, false>(k);
    }
    if (adaptive) rat ? pick_arc<true, true>(k) : pick_arc<true, false>(k);
    else rat ? pick_arc<false, true>(k) : pick_arc<false, false>(k);
    k.surface = ext ? surface_pick<T, kRowExt>(nrm, nt, K) : surface_pick<T, 16>(nrm, nt, K);
    return k;
}

BatchedKernels batched_kernels(bool f64, bool t64, bool nrm, bool nontemporal, int tile_vertices, bool ext, bool arc,
                               bool adaptive, bool rat)
{
    const int K = tile_vertices / kBlock;
    if (f64)
        return t64 ? pick<double, double>(nrm, nontemporal, K, ext, arc, adaptive, rat)
                   : pick<double, float>(nrm, nontemporal, K, ext, arc, adaptive, rat);
    return t64 ? pick<float, double>(nrm, nontemporal, K, ext, arc, adaptive, rat)
               : pick<float, float>(nrm, nontemporal, K, ext, arc, adaptive, rat);
}

}  // namespace sweep
