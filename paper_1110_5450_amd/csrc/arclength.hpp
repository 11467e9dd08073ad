// arclength.hpp -- the arc-length sampling of a path (device functions
// shared by the single-sweep and batched kernels).
//
// Arc length s(u) = integral of |C'| from the start of the domain.  Every
// non-empty knot span is cut into kArcSub equal pieces, each integrated by
// 8-point Gauss-Legendre (one lane per node); one block scans the piece
// lengths into a cumulative table; a group of lanes per u-sample finds the
// piece holding its target length i/(n_u-1) of the total (binary search)
// and solves s(u) = target inside it by Newton's method kept in a bisection
// bracket, the running integral again by 8-point Gauss-Legendre over
// [piece start, u].  The sample parameters and their spans then replace the
// uniform parameter rule for the path.
#pragma once

#include "device_math.hpp"
#include "kernels.hpp"

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

// Piece q = (k - p) * kArcSub + m of span k: its bounds.
__device__ __forceinline__ void piece_bounds(const DCurve& c, int q, int& k, double& lo, double& hi)
{
    k = c.p + q / kArcSub;
    const int m = q % kArcSub;
    const double Uk = knot(c, k), Uk1 = knot(c, k + 1), w = Uk1 - Uk;
    lo = Uk + w * ((double)m / kArcSub);
    hi = m + 1 < kArcSub ? Uk + w * ((double)(m + 1) / kArcSub) : Uk1;
}

// Piece q's length into len[q]: eight lanes per piece (l = the lane's node),
// one Gauss-Legendre node each; the weighted speeds are summed by a
// butterfly over the eight lanes.
template <int P, bool ADAPT>
__device__ __forceinline__ void arc_piece(const DCurve& c, int q, int l, double lam, double* __restrict__ len)
{
    int k;
    double lo, hi;
    piece_bounds(c, q, k, lo, hi);
    if (!(hi > lo)) {
        if (l == 0) len[q] = 0.0;
        return;
    }
    const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
    double part = kGlW[l] * speed_at<P, ADAPT>(c, k, mid + half * kGlX[l], lam);
    part += __shfl_xor(part, 1, 8);
    part += __shfl_xor(part, 2, 8);
    part += __shfl_xor(part, 4, 8);
    if (l == 0) len[q] = half * part;
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
// coarse table in LDS (nc = npc / cstride + 1 entries).
template <int P, bool ADAPT>
__device__ __forceinline__ void arc_param(const DCurve& c, int i, int l, int ns, int npc, int cstride, int nc,
                                          double lam, const double* __restrict__ cum, const double* coarse,
                                          double* __restrict__ su, int* __restrict__ ss)
{
    double u;
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
        const double len = cum[q + 1] - cum[q];
        u = len > 0.0 ? plo + (target - cum[q]) / len * (phi - plo) : plo;
        double blo = plo, bhi = phi;
        const double xl = kGlX[l], wl = kGlW[l];
        // Every lane of the group holds the same u, f and speed (the sums
        // below are butterflies, whose pairwise additions commute), so the
        // group takes every branch together.
        for (int it = 0; it < 40; ++it) {
            const double mid = 0.5 * (plo + u), half = 0.5 * (u - plo);
            const double e = speed_at<P, ADAPT>(c, k, mid + half * xl, lam);
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
        ss[i] = span_of(c, u);
    }
}


// Runtime path degree (one copy per degree, as the single-sweep launches
// select at run time).
template <bool ADAPT>
__device__ __forceinline__ void arc_piece_any(const DCurve& c, int q, int l, double lam, double* __restrict__ len)
{
    switch (c.p) {
    case 1: arc_piece<1, ADAPT>(c, q, l, lam, len); break;
    case 2: arc_piece<2, ADAPT>(c, q, l, lam, len); break;
    case 3: arc_piece<3, ADAPT>(c, q, l, lam, len); break;
    case 4: arc_piece<4, ADAPT>(c, q, l, lam, len); break;
    case 5: arc_piece<5, ADAPT>(c, q, l, lam, len); break;
    case 6: arc_piece<6, ADAPT>(c, q, l, lam, len); break;
    default: arc_piece<7, ADAPT>(c, q, l, lam, len); break;
    }
}
template <bool ADAPT>
__device__ __forceinline__ void arc_param_any(const DCurve& c, int i, int l, int ns, int npc, int cstride, int nc,
                                              double lam, const double* __restrict__ cum, const double* coarse,
                                              double* __restrict__ su, int* __restrict__ ss)
{
    switch (c.p) {
    case 1: arc_param<1, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    case 2: arc_param<2, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    case 3: arc_param<3, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    case 4: arc_param<4, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    case 5: arc_param<5, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    case 6: arc_param<6, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    default: arc_param<7, ADAPT>(c, i, l, ns, npc, cstride, nc, lam, cum, coarse, su, ss); break;
    }
}

// Pieces of an open path's arc-length table.
__host__ __device__ inline int arc_piece_count(int n, int p) { return (n - p) * kArcSub; }

}  // namespace sweep

#pragma clang fp contract(fast)
