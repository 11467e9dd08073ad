// arclength.hpp -- the arc-length sampling of a path (device functions
// shared by the single-sweep and batched kernels).
//
// Arc length s(u) = integral of |C'| from the start of the domain.  Every
// non-empty knot span is cut into kArcSub equal pieces, each integrated by
// 8-point Gauss-Legendre (a wave per span, four nodes per lane); one block
// scans the piece lengths into a cumulative table; a group of lanes per
// u-sample finds the piece holding its target length i/(n_u-1) of the total
// (binary search) and solves s(u) = target inside it by Newton's method
// kept in a bisection bracket, the running integral again by 8-point
// Gauss-Legendre over [piece start, u].  C' of a polynomial path is
// evaluated from a per-span set-up (SpanDeriv) formed once per span or per
// sample.  The sample parameters and their spans then replace the
// uniform parameter rule for the path.
#pragma once

#include "device_math.hpp"
#include "kernels.hpp"
#include "sweep.h"

#pragma clang fp contract(off)

namespace sweep {


constexpr int kArcSub = 32;

// 8-point Gauss-Legendre nodes on [-1, 1] and weights.
static __device__ const double kGlX[8] = {-0.9602898564975362, -0.7966664774136267, -0.525532409916329,
                                   -0.18343464249564978, 0.18343464249564978, 0.525532409916329,
                                   0.7966664774136267,  0.9602898564975362};
static __device__ const double kGlW[8] = {0.10122853629037669, 0.22238103445337434, 0.31370664587788705,
                                   0.36268378337836177, 0.36268378337836177, 0.31370664587788705,
                                   0.22238103445337434, 0.10122853629037669};

// Sampling density at u on span s: |C'| (arc length), and with ADAPT
// |C'| + lam |C' x C''| / |C'|^2 = |C'| (1 + lam kappa), whose integral is
// arc length plus lam times the turning angle (curvature-adaptive sampling).
template <int P, bool ADAPT>
__device__ double speed_at(const DCurve& c, int s, double u, double lam)
{
    V3<double> o[3];
    curve_derivs<P, ADAPT ? 2 : 1>(c, u, s, o);
    const double sp = sqrt(dot(o[1], o[1]));
    if (!ADAPT) return sp;
    const V3<double> cr = cross(o[1], o[2]);
    return sp + (sp > 0.0 ? lam * sqrt(dot(cr, cr)) / (sp * sp) : 0.0);
}

// Weights that extrapolate the degree-7 interpolant of values at the eight
// Gauss-Legendre nodes to the end point +1: the Lagrange basis polynomials of
// the nodes at +1 (computed in extended precision, rounded to double; their
// absolute values sum to 4.5).
static __device__ const double kGlEnd[8] = {-0.032020422845832404, 0.11217721020871642, -0.2208713667044389,
                                     0.3537304181064418,    -0.5126556338013685, 0.7101568903172424,
                                     -0.9912041583117163,   1.5806870630309555};

// C' of a polynomial path on one non-empty span k, set up for evaluation by
// de Boor's algorithm with multiplications only (degree d = p-1):
//   e_t = p (P_{k-p+t+1} - P_{k-p+t}) / (U_{k+t+1} - U_{k-p+t+1}),  t = 0..p-1,
// the control points of C' that act on the span; the reciprocals
//   R_{r,i} = 1 / (U_{k+i+1-r} - U_{k-d+i}),  1 <= r <= i <= d,
// of the denominators of level r of the recursion; and the knots U_{k-d+i},
// i = 0..d+1 (U_k and U_{k+1} among them).  Each of the p + d(d+1)/2 + d + 2
// values is one job, so that a group of lanes forms them together.  Every
// denominator spans an interval that contains the span [U_k, U_{k+1}), so
// none vanishes on a non-empty span (an empty span's quotients are not
// used).
template <int P>
struct SpanDeriv {
    static constexpr int kD = P - 1;
    static constexpr int kNR = kD * (kD + 1) / 2;
    static constexpr int kR = 3 * P;           // R_{r,i} at kR + (i-1) i / 2 + r - 1
    static constexpr int kU = kR + kNR;        // U_{k-d+i} at kU + i, i = 0..d+1
    // the jobs in this order: e_t, R_{r,i}, the knots of i = 1..d (all
    // that the evaluation needs: the first kJobsEval), then U_{k+1}, U_{k-d}
    static constexpr int kJobsEval = P + kNR + kD;
    static constexpr int kJobs = kJobsEval + 2;
    static constexpr int kDoubles = kU + kD + 2;
};
constexpr int kArcSetupMax = SpanDeriv<SWEEP_MAX_DEGREE>::kDoubles;

template <int P>
__device__ __forceinline__ void span_deriv_job(const DCurve& c, int k, int j, double* __restrict__ s)
{
    using S = SpanDeriv<P>;
    constexpr int D = S::kD;
    // every job reads two knots U_a, U_b and forms one quotient (the lanes
    // of a group take one pass instead of one per kind of job): e_t's
    // factor p / (U_b - U_a), R_{r,i} = 1 / (U_b - U_a), or the knot U_b
    int ia, ib, idx = 0;
    double num;
    if (j < P) {
        ia = k - P + j + 1;
        ib = k + j + 1;
        num = (double)P;
    } else if (j < P + S::kNR) {
        idx = j - P;
        int i = 1;
#pragma unroll
        for (int m = 2; m <= D; ++m)
            if (idx >= (m - 1) * m / 2) i = m;
        const int r = idx - (i - 1) * i / 2 + 1;
        ia = k - D + i;
        ib = k + i + 1 - r;
        num = 1.0;
    } else {
        const int m = j - P - S::kNR;
        idx = m < D ? m + 1 : (m == D ? D + 1 : 0);   // knot U_{k-d+idx}
        ia = ib = k - D + idx;
        num = 0.0;
    }
    const double ua = knot(c, ia), ub = knot(c, ib);
    const double f = num / (ub - ua);   // (a knot job's 0 / 0 is not used)
    if (j < P) {
        const V3<double> a = ctrl_pt(c, k - P + j), b = ctrl_pt(c, k - P + j + 1);
        s[3 * j] = f * (b.x - a.x);
        s[3 * j + 1] = f * (b.y - a.y);
        s[3 * j + 2] = f * (b.z - a.z);
    } else if (j < P + S::kNR) {
        s[S::kR + idx] = f;
    } else if (j < S::kJobs) {
        s[S::kU + idx] = ub;
    }
}

// The sampling density (as speed_at) at u on the span set up in s: level r
// of the recursion replaces e_i, i = d..r, by e_{i-1} + a (e_i - e_{i-1}),
// a = (u - U_{k-d+i}) R_{r,i}; e_d is then C'(u).  C'' (adaptive sampling)
// is d R_{d,d} (e_d - e_{d-1}) taken before the last level (R_{d,d} is the
// reciprocal of the span's width).
template <int P, bool ADAPT>
__device__ __forceinline__ double span_speed(const double* __restrict__ s, double u, double lam)
{
    // component-wise with fused multiply-adds: the node values agree with
    // the oracle's to rounding, not bitwise, either way
    using S = SpanDeriv<P>;
    constexpr int D = S::kD;
    double ex[P], ey[P], ez[P];
#pragma unroll
    for (int t = 0; t < P; ++t) {
        ex[t] = s[3 * t];
        ey[t] = s[3 * t + 1];
        ez[t] = s[3 * t + 2];
    }
    double c2x = 0.0, c2y = 0.0, c2z = 0.0;
#pragma unroll
    for (int r = 1; r <= D; ++r) {
        if constexpr (ADAPT && D >= 1) {
            if (r == D) {
                const double f = (double)D * s[S::kR + (D - 1) * D / 2 + D - 1];
                c2x = f * (ex[D] - ex[D - 1]);
                c2y = f * (ey[D] - ey[D - 1]);
                c2z = f * (ez[D] - ez[D - 1]);
            }
        }
#pragma unroll
        for (int i = D; i >= r; --i) {
            const double a = (u - s[S::kU + i]) * s[S::kR + (i - 1) * i / 2 + r - 1];
            ex[i] = fma(a, ex[i] - ex[i - 1], ex[i - 1]);
            ey[i] = fma(a, ey[i] - ey[i - 1], ey[i - 1]);
            ez[i] = fma(a, ez[i] - ez[i - 1], ez[i - 1]);
        }
    }
    const double sp = sqrt(fma(ex[D], ex[D], fma(ey[D], ey[D], ez[D] * ez[D])));
    if (!ADAPT) return sp;
    const double cx = ey[D] * c2z - ez[D] * c2y, cy = ez[D] * c2x - ex[D] * c2z, cz = ex[D] * c2y - ey[D] * c2x;
    return sp + (sp > 0.0 ? lam * sqrt(fma(cx, cx, fma(cy, cy, cz * cz))) / (sp * sp) : 0.0);
}

// Piece q = (k - p) * kArcSub + m of span k: its bounds.
__device__ __forceinline__ void piece_bounds(const DCurve& c, int q, int& k, double& lo, double& hi)
{
    k = c.p + q / kArcSub;
    const int m = q % kArcSub;
    const double Uk = knot(c, k), Uk1 = knot(c, k + 1), w = Uk1 - Uk;
    lo = Uk + w * ((double)m / kArcSub);
    hi = m + 1 < kArcSub ? Uk + w * ((double)(m + 1) / kArcSub) : Uk1;
}

// The kArcSub piece lengths of span index si (span k = p + si) into
// len[si kArcSub ...], by one wave: a polynomial path's span is set up once
// (span_deriv_job, one job per lane, through the wave's LDS slice s), then
// lane l takes four nodes of piece l / 2 (the rule is symmetric: the
// positive nodes, mirrored on even lanes) and the two lanes of a piece add
// their weighted sums.  A rational path (RAT) evaluates each node by
// speed_at.  An empty span's pieces have length 0.
template <int P, bool ADAPT, bool RAT>
__device__ __forceinline__ void arc_span(const DCurve& c, int si, int lane, double lam, double* __restrict__ s,
                                         double* __restrict__ len)
{
    static_assert(2 * kArcSub == 64, "two lanes per piece fill a wave");
    using S = SpanDeriv<P>;
    const int k = c.p + si, m = lane >> 1;
    double Uk, Uk1;
    if (!RAT) {
        // the set-up first: U_k and U_{k+1} are two of its jobs
        if (lane < S::kJobs) span_deriv_job<P>(c, k, lane, s);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        Uk = s[S::kU + S::kD];
        Uk1 = s[S::kU + S::kD + 1];
    } else {
        Uk = knot(c, k);
        Uk1 = knot(c, k + 1);
    }
    const double w = Uk1 - Uk;
    double* out = len + (long long)si * kArcSub;
    if (!(w > 0.0)) {
        if (lane < kArcSub) out[lane] = 0.0;
        return;
    }
    // the piece's bounds as piece_bounds forms them
    const double lo = Uk + w * ((double)m / kArcSub);
    const double hi = m + 1 < kArcSub ? Uk + w * ((double)(m + 1) / kArcSub) : Uk1;
    const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo), sh = (lane & 1) ? half : -half;
    double part = 0.0;
#pragma unroll
    for (int t = 4; t < 8; ++t) {
        const double x = mid + sh * kGlX[t];
        const double e = RAT ? speed_at<P, ADAPT>(c, k, x, lam) : span_speed<P, ADAPT>(s, x, lam);
        part += kGlW[t] * e;
    }
    part += __shfl_xor(part, 1, 64);
    if (!(lane & 1)) out[m] = half * part;
}

// Inclusive scan of the piece lengths into cum[1..npc] (cum[0] = 0) by one
// block of kScanThreads over tiles of kScanTile pieces: a coalesced load of
// the tile into LDS, kScanPer consecutive pieces summed per thread, a block
// scan of the thread sums (wave scans by shuffles, then the 16 wave totals),
// the tile written back through LDS with coalesced stores, and a running
// carry between tiles.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;
// LDS slot of tile entry e: one pad slot after every kScanPer entries, so
// that the threads reading their kScanPer consecutive entries (a stride of
// kScanPer + 1 doubles) spread over the banks (136 KiB in all).
__device__ __forceinline__ int scan_slot(int e) { return e + e / kScanPer; }

// The scan by one block of kScanThreads threads (the block's LDS).
__device__ __forceinline__ void arc_cumsum_block(const double* __restrict__ len, int npc, double* __restrict__ cum)
{
    __shared__ double tile[kScanTile + kScanTile / kScanPer];
    __shared__ double wsum[kScanThreads / 64];
    __shared__ double carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) {
        cum[0] = 0.0;
        carry_s = 0.0;
    }
    for (long long base = 0; base < npc; base += kScanTile) {
        // clamped (always in-bounds) loads, so that all kScanPer are in
        // flight together instead of one conditional load at a time
        double ld[kScanPer];
#pragma unroll
        for (int r = 0; r < kScanPer; ++r) {
            const long long q = base + r * kScanThreads + t;
            ld[r] = len[q < npc ? q : npc - 1];
        }
#pragma unroll
        for (int r = 0; r < kScanPer; ++r) {
            const long long q = base + r * kScanThreads + t;
            tile[scan_slot(r * kScanThreads + t)] = q < npc ? ld[r] : 0.0;
        }
        __syncthreads();
        double v[kScanPer];
#pragma unroll
        for (int r = 0; r < kScanPer; ++r) v[r] = tile[scan_slot(t * kScanPer + r)];
#pragma unroll
        for (int r = 1; r < kScanPer; ++r) v[r] += v[r - 1];
        // inclusive scan of the thread sums within the wave
        double x = v[kScanPer - 1];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        double excl = __shfl_up(x, 1, 64);
        if (lane == 0) excl = 0.0;
        __syncthreads();
        if (t == 0) {
            double run = carry_s;
            for (int k = 0; k < kScanThreads / 64; ++k) {
                const double s = wsum[k];
                wsum[k] = run;
                run += s;
            }
            carry_s = run;
        }
        __syncthreads();
        const double off = wsum[w] + excl;
#pragma unroll
        for (int r = 0; r < kScanPer; ++r) tile[scan_slot(t * kScanPer + r)] = off + v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kScanPer; ++r) {
            const long long q = base + r * kScanThreads + t;
            if (q < npc) cum[q + 1] = tile[scan_slot(r * kScanThreads + t)];
        }
        __syncthreads();   // tile, wsum and carry_s are rewritten by the next tile
    }
}

// Span of parameter u by the standard rule (largest k in [p, nb-1] with
// U_k <= u; the last span at the end of the domain).
__device__ __forceinline__ int span_of(const DCurve& c, double u)
{
    if (u >= knot(c, c.nb)) return c.nb - 1;
    int lo = c.p, hi = c.nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (knot(c, mid) <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Lanes per sample in k_arc_params: one Gauss-Legendre node each.  Newton's
// derivative, the density at the iterate, is extrapolated from the eight
// node values (kGlEnd) instead of a ninth evaluation: its relative error
// (about 1e-12 on a piece of a smooth span) only slows the quadratic
// convergence by that factor, and the root is that of the same
// Gauss-Legendre integral.
constexpr int kArcLanes = 8;

// The piece search starts in a coarse copy of the table in LDS (every
// cstride-th entry, at most kArcCoarseMax of them) and ends with a binary
// search over cstride entries in global memory.
constexpr int kArcCoarseMax = 1024;

__host__ __device__ inline int arc_coarse_stride(int npc)
{
    int cs = 64;
    while (npc / cs + 1 > kArcCoarseMax) cs *= 2;
    return cs;
}

// Sample i's parameter and span (lane l of its kArcLanes group), given the
// coarse table in LDS (nc = npc / cstride + 1 entries).  A polynomial path's
// span is set up once for the iteration by the group (its LDS slice gs); a
// rational path (RAT) evaluates each node by speed_at.
template <int P, bool ADAPT, bool RAT>
__device__ __forceinline__ void arc_param(const DCurve& c, int i, int l, int ns, int npc, int cstride, int nc,
                                          double lam, const double* __restrict__ cum, const double* coarse,
                                          double* __restrict__ gs, double* __restrict__ su, int* __restrict__ ss)
{
    double u;
    int ks = -1;   // the span of the piece holding u (interior samples)
    if (i == 0) {
        u = knot(c, c.p);
    } else if (i == ns - 1) {
        u = knot(c, c.nb);
    } else {
        const double target = ((double)i / (double)(ns - 1)) * cum[npc];
        // last piece with cum[q] <= target: first the last coarse entry
        // with coarse[kc] <= target (coarse[0] = 0 always is), then the
        // pieces up to the next coarse entry
        int klo = 0, khi = nc - 1;
        while (klo < khi) {
            const int mid = (klo + khi + 1) >> 1;
            if (coarse[mid] <= target) klo = mid; else khi = mid - 1;
        }
        int lo = min(klo * cstride, npc - 1), hi = min(klo * cstride + cstride - 1, npc - 1);
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cum[mid] <= target) lo = mid; else hi = mid - 1;
        }
        // the last non-empty piece with cum[q] <= target (pieces of empty
        // spans carry no length; cum is non-decreasing, so stepping back
        // keeps cum[q] <= target)
        int q = lo, k;
        double plo, phi;
        piece_bounds(c, q, k, plo, phi);
        while (q > 0 && !(phi > plo)) piece_bounds(c, --q, k, plo, phi);
        ks = k;
        const double len = cum[q + 1] - cum[q];
        u = len > 0.0 ? plo + (target - cum[q]) / len * (phi - plo) : plo;
        double blo = plo, bhi = phi;
        const double xl = kGlX[l], wl = kGlW[l];
        if (!RAT) {
            for (int j = l; j < SpanDeriv<P>::kJobsEval; j += kArcLanes) span_deriv_job<P>(c, k, j, gs);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // Every lane of the group holds the same u, f and speed (the sums
        // below are butterflies, whose pairwise additions commute), so the
        // group takes every branch together.
        for (int it = 0; it < 40; ++it) {
            const double mid = 0.5 * (plo + u), half = 0.5 * (u - plo);
            const double x = mid + half * xl;
            const double e = RAT ? speed_at<P, ADAPT>(c, k, x, lam) : span_speed<P, ADAPT>(gs, x, lam);
            double part = wl * e, sp = kGlEnd[l] * e;
            part += __shfl_xor(part, 1, kArcLanes);
            sp += __shfl_xor(sp, 1, kArcLanes);
            part += __shfl_xor(part, 2, kArcLanes);
            sp += __shfl_xor(sp, 2, kArcLanes);
            part += __shfl_xor(part, 4, kArcLanes);
            sp += __shfl_xor(sp, 4, kArcLanes);
            part = __shfl(part, 0, kArcLanes);
            sp = __shfl(sp, 0, kArcLanes);
            const double f = cum[q] + half * part - target;
            if (f == 0.0) break;
            if (f > 0.0) bhi = u; else blo = u;
            double un = sp > 0.0 ? u - f / sp : 0.5 * (blo + bhi);
            if (!(un >= blo && un <= bhi)) un = 0.5 * (blo + bhi);
            const double du = fabs(un - u);
            u = un;
            if (du <= 4.0 * 2.220446049250313e-16 * (fabs(u) > 1.0 ? fabs(u) : 1.0)) break;
        }
    }
    if (l == 0) {
        su[i] = u;
        // u stays in its piece, so in [U_ks, U_{ks+1}]: the standard rule
        // gives ks unless u is the span's end
        ss[i] = ks >= 0 && u < knot(c, ks + 1) ? ks : span_of(c, u);
    }
}


// Pieces of an open path's arc-length table.
__host__ __device__ inline int arc_piece_count(int n, int p) { return (n - p) * kArcSub; }

}  // namespace sweep

#pragma clang fp contract(fast)
