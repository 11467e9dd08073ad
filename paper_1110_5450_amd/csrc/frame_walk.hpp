// frame_walk.hpp -- the rotation-minimizing frame over runs of consecutive
// u-samples, one run per thread.
//
// A chunk of kBlock*K samples is handled by one block: thread t owns the run
// of K samples starting at i0 = chunk_base + t*K.  Each thread walks its run
// twice:
//   pass 1: the ordered product A_t = M_{i0+K-1} ... M_{i0} of its step
//           rotations (the lookahead sample i0+K belongs to the next run);
//   pass 2: given the normal r entering its run, the row records of its K
//           samples, carrying r_{i+1} = M_i r_i from sample to sample.
// Between the passes a block exclusive product of the A_t gives each run its
// entering normal.  Per sample that is one matrix product and one
// matrix-vector product instead of a block scan, and the samples are
// evaluated from the control points in both passes (no sample planes in
// memory).  The curve is evaluated through a cursor that keeps the current
// knot span's knots, the reciprocals of its knot differences and its control
// points in registers: consecutive samples mostly share a span.
//
// Tangents: t_i = C'_i/|C'_i|; where C'_i = 0 the tangent of the last earlier
// sample with C' != 0 is carried forward (the first control-polygon leg if
// there is none).  A run whose first sample has C' = 0 takes that tangent
// from an earlier run of the chunk, or from the chunk's entry carry.
#pragma once

#include "frame_common.hpp"

#pragma clang fp contract(off)

namespace sweep {

// A path staged in LDS by the block that walks it (stage_path): the knot
// vector (the given one, or the default one materialised), the control
// points, the weights and, per knot span s, the reciprocals of the knot
// differences of the triangular Cox-de Boor sweep,
//   RT[(s - p) P(P+1)/2 + q(q-1)/2 + j] = 1/(U_{s+j+1} - U_{s-q+j+1}),
// formed by the same operations as the cursor's own (identical values).
struct LdsCurve {
    const double* U;
    const double* X;      // n x 3
    const double* W;      // n weights (rational)
    const double* RT;
    int n, p, closed, nb;
    bool rat, given_knots;
    const double* su;     // arc-length samples (set by the caller), or nullptr
    const int* ss;
};
__device__ __forceinline__ bool is_rational(const DCurve& c) { return c.w != nullptr; }
__device__ __forceinline__ bool is_rational(const LdsCurve& c) { return c.rat; }
__device__ __forceinline__ double knot(const LdsCurve& c, int k) { return c.U[k]; }
__device__ __forceinline__ V3<double> ctrl_pt(const LdsCurve& c, int k)
{
    const int kk = (c.closed && k >= c.n) ? k - c.n : k;
    const double* q = c.X + 3 * kk;
    return {q[0], q[1], q[2]};
}
__device__ __forceinline__ double weight_at(const LdsCurve& c, int k)
{
    return c.W[(c.closed && k >= c.n) ? k - c.n : k];
}
// Span of sample i: as sample_span (integer arithmetic for the default knots,
// else a binary search over the staged vector).
__device__ __forceinline__ int sample_span(const LdsCurve& c, int i, int ns, double u)
{
    if (!c.given_knots) {
        if (c.closed) return c.p + (int)(((long long)c.n * (long long)i) / ns);
        const int s = c.p + (int)(((long long)i * (long long)(c.n - c.p)) / (ns - 1));
        return s < c.n - 1 ? s : c.n - 1;
    }
    if (u >= c.U[c.nb]) return c.nb - 1;
    int lo = c.p, hi = c.nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (c.U[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}
// Reciprocals of span sp's knot differences: formed, or read from the table.
template <int P>
__device__ __forceinline__ void span_recips(const DCurve&, int, const double* Uk, double* rt)
{
#pragma unroll
    for (int q = 1; q <= P; ++q)
#pragma unroll
        for (int j = 0; j < q; ++j) rt[q * (q - 1) / 2 + j] = recip(Uk[P + j] - Uk[P - q + j]);
}
template <int P>
__device__ __forceinline__ void span_recips(const LdsCurve& c, int sp, const double*, double* rt)
{
    const double* q = c.RT + (size_t)(sp - P) * (P * (P + 1) / 2);
#pragma unroll
    for (int e = 0; e < P * (P + 1) / 2; ++e) rt[e] = q[e];
}

// Block-cooperative staging of an open path into lds (lds_path_doubles
// doubles, which the caller guarantees).
template <int P>
__device__ LdsCurve stage_path(const DCurve& g, double* lds)
{
    const int nk = g.nb + g.p + 1;
    double* U = lds;
    double* X = U + nk;
    double* W = X + 3 * g.n;
    double* RT = W + (g.w ? g.n : 0);
    for (int k = threadIdx.x; k < nk; k += kBlock) U[k] = knot(g, k);
    for (int k = threadIdx.x; k < 3 * g.n; k += kBlock) X[k] = g.ctrl[k];
    if (g.w)
        for (int k = threadIdx.x; k < g.n; k += kBlock) W[k] = g.w[k];
    __syncthreads();
    constexpr int NR = P * (P + 1) / 2;
    for (int k = threadIdx.x; k < g.nb - P; k += kBlock) {
        const int sp = P + k;
#pragma unroll
        for (int q = 1; q <= P; ++q)
#pragma unroll
            for (int j = 0; j < q; ++j) RT[k * NR + q * (q - 1) / 2 + j] = recip(U[sp + 1 + j] - U[sp + 1 - q + j]);
    }
    __syncthreads();
    return LdsCurve{U, X, W, RT, g.n, g.p, g.closed, g.nb, g.w != nullptr, g.knots != nullptr, nullptr, nullptr};
}

// Open curve evaluated at samples of increasing index.  Knot span data are
// loaded when the span changes: the 2P knots U_{s-P+1} .. U_{s+P}, the
// reciprocals of the knot differences used by the triangular Cox-de Boor
// sweep and by the derivative control nets, the P+1 control points and (for a
// rational curve) their weights.
template <int P>
struct PathCursor {
    int s = -1;
    double ua, ub;                     // open curve: parameter range [U_p, U_n]
    double Uk[2 * P];
    double rt[P * (P + 1) / 2];        // 1/(U_{s+j+1} - U_{s-q+j+1}), q = 1..P, j < q, at q(q-1)/2 + j
    double f1[P > 0 ? P : 1];          // P/(U_{s+j+1} - U_{s-P+j+1})
    double f2[P > 1 ? P - 1 : 1];      // (P-1)/(U_{s+j+1} - U_{s-P+j+2})
    double f3[P > 2 ? P - 2 : 1];      // (P-2)/(U_{s+j+1} - U_{s-P+j+3})
    V3<double> Pt[P + 1];
    double w[P + 1];

    template <int ND, class C>
    __device__ __forceinline__ void load(const C& c, int sp)
    {
        s = sp;
#pragma unroll
        for (int m = 0; m < 2 * P; ++m) Uk[m] = knot(c, sp - P + 1 + m);
        span_recips<P>(c, sp, Uk, rt);
        // the derivative nets' factors reuse the reciprocals of the same
        // knot differences (q = P, P-1, P-2 above)
        if (ND >= 1) {
#pragma unroll
            for (int j = 0; j < P; ++j) f1[j] = (double)P * rt[P * (P - 1) / 2 + j];
        }
        if (ND >= 2 && P >= 2) {
#pragma unroll
            for (int j = 0; j + 1 < P; ++j) f2[j] = (double)(P - 1) * rt[(P - 1) * (P - 2) / 2 + j];
        }
        if (ND >= 3 && P >= 3) {
#pragma unroll
            for (int j = 0; j + 2 < P; ++j) f3[j] = (double)(P - 2) * rt[(P - 2) * (P - 3) / 2 + j];
        }
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            Pt[j] = ctrl_pt(c, sp - P + j);
            w[j] = is_rational(c) ? weight_at(c, sp - P + j) : 1.0;
            if (is_rational(c)) Pt[j] = w[j] * Pt[j];   // homogeneous point of a rational curve
        }
    }

    // The range ends of the uniform samples (open curves), read once.
    template <class C>
    __device__ __forceinline__ void start(const C& c)
    {
        ua = c.closed ? 0.0 : knot(c, c.p);
        ub = c.closed ? 0.0 : knot(c, c.n);
    }

    // C and its derivatives up to order ND at sample i of ns.  The samples'
    // parameters and spans are given (arc-length sampling, c.su and c.ss),
    // or the uniform samples are formed here with the rounding of
    // sample_param.
    template <int ND, class C>
    __device__ __forceinline__ void eval(const C& c, int i, int ns, V3<double>* out)
    {
        double u;
        int sp;
        if (c.su) {
            u = c.su[i];
            sp = c.ss[i];
        } else {
            if (c.closed) {
                u = (double)c.p + (double)((long long)c.n * (long long)i) / (double)ns;
            } else if (i == ns - 1) {
                u = ub;
            } else {
                const double f = (double)i / (double)(ns - 1);
                const double w = ub - ua;
                const double g = w * f;
                u = ua + g;
            }
            if (s < 0) {
                sp = sample_span(c, i, ns, u);
            } else {
                // samples increase: advance from the cached span while the
                // next knot is <= u (the last span at the domain's end)
                sp = s;
                double above = Uk[P];
                while (sp < c.nb - 1 && above <= u) {
                    ++sp;
                    above = knot(c, sp + 1);
                }
            }
        }
        if (sp != s) load<ND>(c, sp);
        // basis values of degrees P, P-1, P-2, P-3 (one triangular sweep)
        double B[P + 1];
        double D1[P > 0 ? P : 1];
        double D2[P > 1 ? P - 1 : 1];
        double D3[P > 2 ? P - 2 : 1];
        B[0] = 1.0;
        if (P - 1 == 0) D1[0] = 1.0;
        if (P - 2 == 0) D2[0] = 1.0;
        if (ND >= 3 && P - 3 == 0) D3[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= P; ++q) {
            double nb_[P + 1];
            double carry = 0.0;
#pragma unroll
            for (int j = 0; j < q; ++j) {
                const double lo = Uk[P - q + j], hi = Uk[P + j];
                const double tmp = B[j] * rt[q * (q - 1) / 2 + j];
                nb_[j] = fma(hi - u, tmp, carry);
                carry = (u - lo) * tmp;
            }
            nb_[q] = carry;
#pragma unroll
            for (int j = 0; j <= q; ++j) B[j] = nb_[j];
            if (q == P - 1) {
#pragma unroll
                for (int j = 0; j <= q; ++j) D1[j] = B[j];
            }
            if (q == P - 2) {
#pragma unroll
                for (int j = 0; j <= q; ++j) D2[j] = B[j];
            }
            if (ND >= 3 && q == P - 3) {
#pragma unroll
                for (int j = 0; j <= q; ++j) D3[j] = B[j];
            }
        }
        // Sums over the span's control points.  For a rational curve the
        // cached points are the homogeneous w P and the weight sums run
        // beside them; then the quotient rule (NURBS Book ch. 4).
        const bool rat = is_rational(c);
        V3<double> C0 = mk(0.0, 0.0, 0.0);
        double W0 = 0.0;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            C0 = fmadd(B[j], Pt[j], C0);
            if (rat) W0 = fma(B[j], w[j], W0);
        }
        const double iW = rat ? 1.0 / W0 : 1.0;
        if (rat) C0 = iW * C0;
        out[0] = C0;
        if (ND >= 1) {
            V3<double> Q1[P > 0 ? P : 1];
            double q1[P > 0 ? P : 1];
            V3<double> C1 = mk(0.0, 0.0, 0.0);
            double W1 = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                Q1[j] = f1[j] * (Pt[j + 1] - Pt[j]);
                C1 = fmadd(D1[j], Q1[j], C1);
                if (rat) {
                    q1[j] = f1[j] * (w[j + 1] - w[j]);
                    W1 = fma(D1[j], q1[j], W1);
                }
            }
            if (rat) C1 = iW * fmadd(-W1, C0, C1);
            out[1] = C1;
            if (ND >= 2) {
                V3<double> R2[P > 1 ? P - 1 : 1];
                double r2[P > 1 ? P - 1 : 1];
                V3<double> C2 = mk(0.0, 0.0, 0.0);
                double W2 = 0.0;
#pragma unroll
                for (int j = 0; j + 1 < P; ++j) {
                    R2[j] = f2[j] * (Q1[j + 1] - Q1[j]);
                    C2 = fmadd(D2[j], R2[j], C2);
                    if (rat) {
                        r2[j] = f2[j] * (q1[j + 1] - q1[j]);
                        W2 = fma(D2[j], r2[j], W2);
                    }
                }
                if (rat) C2 = iW * fmadd(-W2, C0, fmadd(-2.0 * W1, C1, C2));
                out[2] = C2;
                if (ND >= 3) {
                    V3<double> C3 = mk(0.0, 0.0, 0.0);
                    double W3 = 0.0;
#pragma unroll
                    for (int j = 0; j + 2 < P; ++j) {
                        C3 = fmadd(D3[j], f3[j] * (R2[j + 1] - R2[j]), C3);
                        if (rat) W3 = fma(D3[j], f3[j] * (r2[j + 1] - r2[j]), W3);
                    }
                    if (rat) C3 = iW * fmadd(-W3, C0, fmadd(-3.0 * W2, C1, fmadd(-3.0 * W1, C2, C3)));
                    out[3] = C3;
                }
            }
        }
    }
};

// Resolved tangent: C'/|C'| where C' != 0, else the carried tangent.
__device__ __forceinline__ bool speed_nonzero(V3<double> d) { return dot(d, d) > 0.0; }

// Pass 1 of one run: A = M_{i_end-1} ... M_{i0} over the steps i -> i+1 with
// i0 <= i < min(i0 + K, n_u - 1).  t_in is the tangent carried into the run
// (used when C'_{i0} = 0).  Also returns the run's resolved first tangent,
// the last sample of the run (i0 .. i0+K-1) with C' != 0 (-1 if none) and its
// tangent, and whether C'_{i0} != 0.
template <int P, class F>
struct RunInfo {
    M3<F> A;
    V3<double> t_first;
    V3<double> t_last_valid;
    int last_valid;
    bool first_valid;
};

template <int P, class F, class C>
__device__ __forceinline__ RunInfo<P, F> run_product(const C& path, int n_u, int i0, int K,
                                                          V3<double> t_in)
{
    RunInfo<P, F> R;
    R.A = ident<F>();
    R.last_valid = -1;
    R.first_valid = false;
    R.t_first = t_in;
    R.t_last_valid = t_in;
    if (i0 >= n_u) return R;
    PathCursor<P> cur;
    cur.start(path);
    V3<double> o[2];
    cur.template eval<1>(path, i0, n_u, o);
    V3<double> xa = o[0];
    R.first_valid = speed_nonzero(o[1]);
    V3<double> ta = R.first_valid ? unit_of(o[1]) : t_in;
    R.t_first = ta;
    if (R.first_valid) { R.last_valid = i0; R.t_last_valid = ta; }
    const int iend = min(i0 + K, n_u);   // the run's own samples are i0 .. iend-1
#pragma nounroll
    for (int i = i0; i + 1 < n_u && i < iend; ++i) {
        cur.template eval<1>(path, i + 1, n_u, o);
        const bool vb = speed_nonzero(o[1]);
        const V3<double> tb = vb ? unit_of(o[1]) : ta;
        if (vb && i + 1 < iend) { R.last_valid = i + 1; R.t_last_valid = tb; }
        apply_step(make_step<F>(cvt<F>(o[0] - xa), cvt<F>(ta), cvt<F>(tb)), R.A);
        xa = o[0];
        ta = tb;
    }
    return R;
}

// Pass 2 of one run: row records of samples i0 .. min(i0+K, n_u)-1, given the
// resolved tangent at i0 (t_first) and the normal entering the run (r, in the
// frame precision).  `row(i, x, t, C', C'', r)` writes one record (ND = 2, or
// 3 with the third derivative in o[3] for the Frenet mode).
template <int P, int ND, class F, class C, class RowFn>
__device__ __forceinline__ void run_rows(const C& path, int n_u, int i0, int K, V3<double> t_first, V3<F> r,
                                         RowFn&& row)
{
    if (i0 >= n_u) return;
    // an opaque copy of the start index: keeps the compiler from sharing the
    // first sample's evaluation with pass 1 across the block scan between the
    // passes (that kept pass 1's registers live through the scan)
    asm volatile("" : "+v"(i0));
    PathCursor<P> cur;
    cur.start(path);
    V3<double> a[ND + 1], b[ND + 1];
    cur.template eval<ND>(path, i0, n_u, a);
    V3<double> ta = t_first;
    const int iend = min(i0 + K, n_u);
#pragma nounroll
    for (int i = i0; i < iend; ++i) {
        // The next sample is evaluated before this sample's record is
        // stored: the loads it may issue (knot span data) then wait only for
        // the stores of the previous record, not for these (the vector
        // memory counter retires loads and stores in issue order).
        const bool more = i + 1 < n_u;
        if (more) cur.template eval<ND>(path, i + 1, n_u, b);
        row(i, a, ta, r);
        if (!more) break;
        const V3<double> tb = speed_nonzero(b[1]) ? unit_of(b[1]) : ta;
        r = apply_step(make_step<F>(cvt<F>(b[0] - a[0]), cvt<F>(ta), cvt<F>(tb)), r);
        ta = tb;
#pragma unroll
        for (int d = 0; d <= ND; ++d) a[d] = b[d];
    }
}

// Row writer of the plain row records.
template <class F, class T>
struct PlainRows {
    T* rows;
    int reorth;
    __device__ __forceinline__ void operator()(int i, const V3<double>* a, V3<double> t, V3<F> r) const
    {
        write_row<F, T>(a[0], t, r, a[1], a[2], reorth, rows + 16 * (size_t)i);
    }
};

// Row writer of the extended records (Frenet frame mode and/or a sweep law).
template <class F, class T>
struct ExtRows {
    T* rows;
    int reorth, frenet, has_law, n_u;
    DCurve law;
    double du_scale;
    __device__ __forceinline__ void operator()(int i, const V3<double>* a, V3<double> t, V3<F> r) const
    {
        const LawSample lw = law_at(has_law ? &law : nullptr, i, n_u, du_scale);
        write_row_ext<F, T>(a[0], t, r, a[1], a[2], a[3], frenet, lw, reorth, rows + kRowExt * (size_t)i);
    }
};

// Chunk-level pass 1 by one block: every thread's run product with the
// tangent carries resolved inside the chunk.  entry_known: the tangent
// carried into the chunk (t_entry) is known (chunk 0: the fallback; later
// chunks: from the chunks before).  Returns false (block-uniform) when the
// chunk's first sample has C' = 0 and the entry carry is not known: the
// products are then not formed.  Also gives the chunk's last sample with
// C' != 0 (chunk_lv, -1 if none) and its tangent (chunk_tl).
struct ChunkWalkLds {
    double tl[3][kBlock];
    int ii[kWaves];
    int flag;
};

template <int P, class F, class C>
__device__ bool chunk_products(const C& path, int n_u, int base, int K, bool entry_known, V3<double> t_entry,
                               ChunkWalkLds& L, RunInfo<P, F>& R, int& chunk_lv, V3<double>& chunk_tl)
{
    const int i0 = base + threadIdx.x * K;
    bool ok = true, redo = false;
    V3<double> tc = t_entry;
    // one call site of run_product: the second pass only re-walks runs whose
    // first sample has C' = 0, with the carry resolved in the first
#pragma nounroll
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 0 || redo) R = run_product<P, F>(path, n_u, i0, K, tc);
        if (pass == 1) break;
        L.tl[0][threadIdx.x] = R.t_last_valid.x;
        L.tl[1][threadIdx.x] = R.t_last_valid.y;
        L.tl[2][threadIdx.x] = R.t_last_valid.z;
        int total;
        const int src = block_exclusive_max(R.last_valid, L.ii, total);   // has barriers: tl is visible after it
        chunk_lv = total;
        chunk_tl = t_entry;
        if (total >= 0) {
            const int owner = (total - base) / K;
            chunk_tl = mk(L.tl[0][owner], L.tl[1][owner], L.tl[2][owner]);
        }
        // the chunk's first sample (thread 0's) decides whether the carries resolve
        if (threadIdx.x == 0) L.flag = (i0 < n_u && !R.first_valid && !entry_known) ? 1 : 0;
        __syncthreads();
        ok = L.flag == 0;
        redo = ok && i0 < n_u && !R.first_valid;
        if (redo && src >= 0) {
            // carried tangent from an earlier run of the chunk, else the entry
            const int owner = (src - base) / K;
            tc = mk(L.tl[0][owner], L.tl[1][owner], L.tl[2][owner]);
        }
        __syncthreads();
    }
    return ok;
}

}  // namespace sweep

#pragma clang fp contract(fast)
