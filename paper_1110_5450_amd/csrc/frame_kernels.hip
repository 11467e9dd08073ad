// frame_kernels.hip -- curve sampling and the rotation-minimizing frame of a
// single sweep as a three-pass parallel prefix product of 3x3 rotations.
//
// Pass A  k_path_samples    C, C', C'' at every u-sample (FP64, SoA planes);
//                           per chunk the last sample with C' != 0.
//         k_profile_table   S, S' at every v-sample in the output precision.
// Pass B  k_frame_reduce    per chunk of kChunk samples: tangents (degenerate
//                           ones carried from the last valid sample), step
//                           rotations M_i, and their ordered product A_b.
// Pass C  k_frame_carry     one block: exclusive ordered product of the A_b
//                           applied to r_0, giving the normal entering chunk b.
// Pass D  k_frame_apply     per chunk: block exclusive product of the thread
//                           products, then each thread walks its samples,
//                           re-orthonormalises and writes the row table
//                           (x, r, s, t, |C'|, a, b) in the output precision.
//
// The step rotations are rebuilt in pass D from the same inputs with the
// same code as in pass B, so both passes see bitwise identical M_i.
#include "device_math.hpp"
#include "kernels.hpp"

namespace sweep {

// Samples per thread in the scan passes and samples per chunk.
constexpr int kSpt = 4;
constexpr int kChunk = kBlock * kSpt;

// smp layout: plane c (0..8 = x, C', C'') of n_u doubles.
__device__ __forceinline__ V3<double> smp_get(const double* __restrict__ smp, size_t n_u, int plane, int i)
{
    return {smp[(size_t)(3 * plane) * n_u + i], smp[(size_t)(3 * plane + 1) * n_u + i],
            smp[(size_t)(3 * plane + 2) * n_u + i]};
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_path_samples(DCurve path, int n_u, double* __restrict__ smp,
                                                         int* __restrict__ chunk_lv, double* __restrict__ fallback_t)
{
    __shared__ int lds[kWaves];
    const size_t nu = (size_t)n_u;
    int best = -1;
    for (int k = 0; k < kSpt; ++k) {
        const int i = blockIdx.x * kChunk + k * kBlock + threadIdx.x;
        if (i < n_u) {
            V3<double> o[3];
            curve_derivs<P, 2>(path, sample_param(path, i, n_u), o);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                smp[(size_t)(3 * d) * nu + i] = o[d].x;
                smp[(size_t)(3 * d + 1) * nu + i] = o[d].y;
                smp[(size_t)(3 * d + 2) * nu + i] = o[d].z;
            }
            if (dot(o[1], o[1]) > 0.0) best = max(best, i);
        }
    }
    int total;
    block_exclusive_max(best, lds, total);
    if (threadIdx.x == 0) chunk_lv[blockIdx.x] = total;
    // Unit direction of the first nonzero control-polygon leg (used only when
    // C'(u_0) = 0), else e_z.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        V3<double> t = mk(0.0, 0.0, 1.0);
        for (int k = 0; k + 1 < path.n; ++k) {
            const V3<double> d = ctrl_pt(path, k + 1) - ctrl_pt(path, k);
            const double L2 = dot(d, d);
            if (L2 > 0.0) { t = divs(d, sqrt(L2)); break; }
        }
        fallback_t[0] = t.x; fallback_t[1] = t.y; fallback_t[2] = t.z;
    }
}

// Profile table, 8 values per v-sample: S (3), S' (3), 0, 0.
template <class T, int P>
__global__ __launch_bounds__(kBlock) void k_profile_table(DCurve prof, int n_v, T* __restrict__ tab)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n_v) return;
    V3<double> o[2];
    curve_derivs<P, 1>(prof, sample_param(prof, j, n_v), o);
    T* q = tab + 8 * (size_t)j;
    q[0] = (T)o[0].x; q[1] = (T)o[0].y; q[2] = (T)o[0].z;
    q[3] = (T)o[1].x; q[4] = (T)o[1].y; q[5] = (T)o[1].z;
    q[6] = T(0); q[7] = T(0);
}

// Shared by passes B and D: for the thread's kSpt consecutive samples
// i0..i0+kSpt-1 (and the following sample) resolve the tangents and build
// the step rotations M_i (identity past the last step).
struct ThreadSamples {
    V3<double> x[kSpt + 1];
    V3<double> t[kSpt + 1];
};

__device__ __forceinline__ V3<double> unit_tangent(const double* __restrict__ smp, size_t nu, int i)
{
    const V3<double> d = smp_get(smp, nu, 1, i);
    return divs(d, sqrt(dot(d, d)));
}

__device__ void load_thread_samples(const double* __restrict__ smp, int n_u, const int* __restrict__ chunk_lv,
                                    const double* __restrict__ fallback_t, int* lds_i, ThreadSamples& ts)
{
    const size_t nu = (size_t)n_u;
    const int i0 = blockIdx.x * kChunk + threadIdx.x * kSpt;
    // last valid sample before this chunk
    int carry = -1;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) carry = max(carry, chunk_lv[b]);
    int dummy;
    {
        // block max of carry (exclusive scan used as a reduction)
        int e = block_exclusive_max(carry, lds_i, dummy);
        (void)e;
        carry = dummy;
    }
    bool valid[kSpt + 1];
    int local = -1;
#pragma unroll
    for (int k = 0; k <= kSpt; ++k) {
        const int i = i0 + k;
        valid[k] = false;
        if (i < n_u) {
            ts.x[k] = smp_get(smp, nu, 0, i);
            const V3<double> d = smp_get(smp, nu, 1, i);
            valid[k] = dot(d, d) > 0.0;
            if (k < kSpt && valid[k]) local = i;
        } else {
            ts.x[k] = mk(0.0, 0.0, 0.0);
        }
    }
    int total;
    int lv = max(carry, block_exclusive_max(local, lds_i, total));
    const V3<double> fb = mk(fallback_t[0], fallback_t[1], fallback_t[2]);
#pragma unroll
    for (int k = 0; k <= kSpt; ++k) {
        const int i = i0 + k;
        if (i < n_u && valid[k]) {
            ts.t[k] = unit_tangent(smp, nu, i);
            if (k < kSpt) lv = i;
        } else {
            ts.t[k] = lv >= 0 ? unit_tangent(smp, nu, lv) : fb;
        }
    }
}

template <class F>
__device__ __forceinline__ void thread_steps(const ThreadSamples& ts, int i0, int n_u, M3<F>* M, M3<F>& prod)
{
    prod = ident<F>();
#pragma unroll
    for (int k = 0; k < kSpt; ++k) {
        const int i = i0 + k;
        if (i + 1 < n_u) {
            const V3<double> v1 = ts.x[k + 1] - ts.x[k];
            step_matrix<F>(cvt<F>(v1), cvt<F>(ts.t[k]), cvt<F>(ts.t[k + 1]), M[k]);
        } else {
            M[k] = ident<F>();
        }
        prod = mul(M[k], prod);
    }
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_frame_reduce(const double* __restrict__ smp, int n_u,
                                                         const int* __restrict__ chunk_lv,
                                                         const double* __restrict__ fallback_t, F* __restrict__ agg)
{
    __shared__ int lds_i[kWaves];
    __shared__ M3<F> lds_m[kWaves];
    ThreadSamples ts;
    load_thread_samples(smp, n_u, chunk_lv, fallback_t, lds_i, ts);
    M3<F> M[kSpt], prod, total;
    thread_steps<F>(ts, blockIdx.x * kChunk + threadIdx.x * kSpt, n_u, M, prod);
    block_exclusive_product<F>(prod, lds_m, total);
    if (threadIdx.x < 9) agg[9 * (size_t)blockIdx.x + threadIdx.x] = total.m[threadIdx.x];
}

// One block: r_in[b] = (A_{b-1} ... A_0) r_0.  r_0 from the resolved t_0 by
// the initial-normal rule.  Also writes r_0 (3) after the n_chunks vectors.
template <class F>
__global__ __launch_bounds__(kBlock) void k_frame_carry(const F* __restrict__ agg, int n_chunks,
                                                        const double* __restrict__ smp, int n_u,
                                                        const double* __restrict__ fallback_t,
                                                        InitialNormal n0, F* __restrict__ r_in)
{
    __shared__ M3<F> lds_m[kWaves];
    // resolved t_0
    V3<double> t0;
    {
        const V3<double> d = smp_get(smp, (size_t)n_u, 1, 0);
        const double L2 = dot(d, d);
        t0 = L2 > 0.0 ? divs(d, sqrt(L2)) : mk(fallback_t[0], fallback_t[1], fallback_t[2]);
    }
    V3<double> r0d;
    bool done = false;
    if (n0.enabled) {
        const V3<double> n = mk(n0.v[0], n0.v[1], n0.v[2]);
        const V3<double> q = n - dot(n, t0) * t0;
        const double L = sqrt(dot(q, q));
        if (L > 1e-8) { r0d = divs(q, L); done = true; }
    }
    if (!done) r0d = axis_normal(t0);
    const V3<F> r0 = cvt<F>(r0d);
    M3<F> running = ident<F>();
    for (int base = 0; base < n_chunks; base += kBlock * kSpt) {
        M3<F> A[kSpt];
        M3<F> prod = ident<F>();
        const int c0 = base + threadIdx.x * kSpt;
#pragma unroll
        for (int k = 0; k < kSpt; ++k) {
            const int c = c0 + k;
            if (c < n_chunks) {
#pragma unroll
                for (int e = 0; e < 9; ++e) A[k].m[e] = agg[9 * (size_t)c + e];
            } else {
                A[k] = ident<F>();
            }
            prod = mul(A[k], prod);
        }
        M3<F> total;
        M3<F> ex = mul(block_exclusive_product<F>(prod, lds_m, total), running);
#pragma unroll
        for (int k = 0; k < kSpt; ++k) {
            const int c = c0 + k;
            if (c < n_chunks) {
                const V3<F> r = apply(ex, r0);
                r_in[3 * (size_t)c] = r.x; r_in[3 * (size_t)c + 1] = r.y; r_in[3 * (size_t)c + 2] = r.z;
            }
            ex = mul(A[k], ex);
        }
        running = mul(total, running);
    }
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
    ThreadSamples ts;
    load_thread_samples(smp, n_u, chunk_lv, fallback_t, lds_i, ts);
    const int i0 = blockIdx.x * kChunk + threadIdx.x * kSpt;
    M3<F> M[kSpt], prod, total;
    thread_steps<F>(ts, i0, n_u, M, prod);
    const M3<F> ex = block_exclusive_product<F>(prod, lds_m, total);
    V3<F> r = apply(ex, mk(r_in[3 * (size_t)blockIdx.x], r_in[3 * (size_t)blockIdx.x + 1], r_in[3 * (size_t)blockIdx.x + 2]));
#pragma unroll
    for (int k = 0; k < kSpt; ++k) {
        const int i = i0 + k;
        if (i >= n_u) break;
        const V3<F> t = cvt<F>(ts.t[k]);
        V3<F> rr = r;
        if (reorth) {
            const V3<F> q = rr - dot(rr, t) * t;
            rr = divs(q, (F)sqrt(dot(q, q)));
        }
        const V3<F> s = cross(t, rr);
        const V3<double> C1 = smp_get(smp, nu, 1, i);
        const V3<double> C2 = smp_get(smp, nu, 2, i);
        const double L = sqrt(dot(C1, C1));
        F a = F(0), b = F(0);
        if (L > 0.0) {
            const V3<F> c2 = cvt<F>(C2);
            a = dot(rr, c2) / (F)L;
            b = dot(s, c2) / (F)L;
        }
        T* q = rows + 16 * (size_t)i;
        q[0] = (T)ts.x[k].x; q[1] = (T)ts.x[k].y; q[2] = (T)ts.x[k].z;
        q[3] = (T)rr.x; q[4] = (T)rr.y; q[5] = (T)rr.z;
        q[6] = (T)s.x; q[7] = (T)s.y; q[8] = (T)s.z;
        q[9] = (T)t.x; q[10] = (T)t.y; q[11] = (T)t.z;
        q[12] = (T)L; q[13] = (T)a; q[14] = (T)b; q[15] = T(0);
        r = apply(M[k], r);
    }
}

// Default knots: periodic U_k = k; clamped uniform 0 (k <= p), 1 (k >= n),
// else (k-p)/(n-p) as one correctly rounded division.
__global__ __launch_bounds__(kBlock) void k_fill_knots(double* __restrict__ U, int n, int p, int closed)
{
    const int nk = (closed ? n + p : n) + p + 1;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < nk; k += gridDim.x * kBlock) {
        double v;
        if (closed) v = (double)k;
        else if (k <= p) v = 0.0;
        else if (k >= n) v = 1.0;
        else v = (double)(k - p) / (double)(n - p);
        U[k] = v;
    }
}

// ------------------------------------------------------------- launchers

hipError_t launch_fill_knots(double* U, int n, int p, int closed, hipStream_t st)
{
    const int nk = (closed ? n + p : n) + p + 1;
    const int grid = (nk + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill_knots, dim3(grid < 64 ? grid : 64), dim3(kBlock), 0, st, U, n, p, closed);
    return hipGetLastError();
}

hipError_t launch_path_samples(const DCurve& path, int n_u, double* smp, int* chunk_lv, double* fallback_t,
                               hipStream_t st)
{
    const int nc = (n_u + kChunk - 1) / kChunk;
#define SWEEP_CASE(P) \
    case P: hipLaunchKernelGGL(k_path_samples<P>, dim3(nc), dim3(kBlock), 0, st, path, n_u, smp, chunk_lv, fallback_t); break;
    switch (path.p) {
        SWEEP_CASE(1) SWEEP_CASE(2) SWEEP_CASE(3) SWEEP_CASE(4) SWEEP_CASE(5) SWEEP_CASE(6) SWEEP_CASE(7)
    default: return hipErrorInvalidValue;
    }
#undef SWEEP_CASE
    return hipGetLastError();
}

template <class T>
hipError_t launch_profile_table(const DCurve& prof, int n_v, T* tab, hipStream_t st)
{
    const dim3 grid((n_v + kBlock - 1) / kBlock);
#define SWEEP_CASE(P) \
    case P: hipLaunchKernelGGL((k_profile_table<T, P>), grid, dim3(kBlock), 0, st, prof, n_v, tab); break;
    switch (prof.p) {
        SWEEP_CASE(1) SWEEP_CASE(2) SWEEP_CASE(3) SWEEP_CASE(4) SWEEP_CASE(5) SWEEP_CASE(6) SWEEP_CASE(7)
    default: return hipErrorInvalidValue;
    }
#undef SWEEP_CASE
    return hipGetLastError();
}
template hipError_t launch_profile_table<float>(const DCurve&, int, float*, hipStream_t);
template hipError_t launch_profile_table<double>(const DCurve&, int, double*, hipStream_t);

template <class F, class T>
hipError_t launch_frame(const double* smp, int n_u, const int* chunk_lv, const double* fallback_t,
                        InitialNormal n0, int reorth, F* agg, F* r_in, T* rows, hipStream_t st)
{
    const int nc = (n_u + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_frame_reduce<F>, dim3(nc), dim3(kBlock), 0, st, smp, n_u, chunk_lv, fallback_t, agg);
    hipLaunchKernelGGL(k_frame_carry<F>, dim3(1), dim3(kBlock), 0, st, agg, nc, smp, n_u, fallback_t, n0, r_in);
    hipLaunchKernelGGL((k_frame_apply<F, T>), dim3(nc), dim3(kBlock), 0, st, smp, n_u, chunk_lv, fallback_t, r_in,
                       reorth, rows);
    return hipGetLastError();
}
template hipError_t launch_frame<double, float>(const double*, int, const int*, const double*, InitialNormal, int,
                                                double*, double*, float*, hipStream_t);
template hipError_t launch_frame<double, double>(const double*, int, const int*, const double*, InitialNormal, int,
                                                 double*, double*, double*, hipStream_t);
template hipError_t launch_frame<float, float>(const double*, int, const int*, const double*, InitialNormal, int,
                                               float*, float*, float*, hipStream_t);
template hipError_t launch_frame<float, double>(const double*, int, const int*, const double*, InitialNormal, int,
                                                float*, float*, double*, hipStream_t);

int frame_chunk_size() { return kChunk; }

}  // namespace sweep
