// arclength_kernels.hip -- arc-length sampling of the path and the grid's
// triangle list.
//
// Arc length s(u) = integral of |C'| from the start of the domain.  Every
// non-empty knot span is cut into kArcSub equal pieces, each integrated by
// 8-point Gauss-Legendre (k_arc_pieces, one lane per node); one block scans
// the piece lengths into a cumulative table (k_arc_cumsum); a group of
// lanes per u-sample finds the piece holding its target length i/(n_u-1) of
// the total (binary search) and solves s(u) = target inside it by Newton's
// method kept in a bisection bracket, the running integral again by
// 8-point Gauss-Legendre over [piece start, u] (k_arc_params).  The sample
// parameters and their spans then replace the uniform parameter rule for
// the path.
#include "device_math.hpp"
#include "kernels.hpp"
#include "surface_common.hpp"

#pragma clang fp contract(off)

namespace sweep {

constexpr int kArcSub = 32;

// 8-point Gauss-Legendre nodes on [-1, 1] and weights.
__device__ const double kGlX[8] = {-0.9602898564975362, -0.7966664774136267, -0.525532409916329,
                                   -0.18343464249564978, 0.18343464249564978, 0.525532409916329,
                                   0.7966664774136267,  0.9602898564975362};
__device__ const double kGlW[8] = {0.10122853629037669, 0.22238103445337434, 0.31370664587788705,
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
__device__ const double kGlEnd[8] = {-0.032020422845832404, 0.11217721020871642, -0.2208713667044389,
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

// Eight lanes per piece, one Gauss-Legendre node each; the weighted speeds
// are summed by a butterfly over the eight lanes.
template <int P, bool ADAPT>
__global__ __launch_bounds__(kBlock) void k_arc_pieces(DCurve c, int npc, double lam, double* __restrict__ len)
{
    const long long g = ((long long)blockIdx.x * kBlock + threadIdx.x) >> 3;
    const int l = threadIdx.x & 7;
    if (g >= npc) return;   // whole 8-lane groups leave together
    const int q = (int)g;
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

__global__ __launch_bounds__(kScanThreads) void k_arc_cumsum(const double* __restrict__ len, int npc,
                                                             double* __restrict__ cum)
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

static int arc_coarse_stride(int npc)
{
    int cs = 64;
    while (npc / cs + 1 > kArcCoarseMax) cs *= 2;
    return cs;
}

template <int P, bool ADAPT>
__global__ __launch_bounds__(kBlock) void k_arc_params(DCurve c, int ns, int npc, int cstride, double lam,
                                                       const double* __restrict__ cum, double* __restrict__ su,
                                                       int* __restrict__ ss)
{
    __shared__ double coarse[kArcCoarseMax];
    const int nc = npc / cstride + 1;   // coarse[k] = cum[k cstride], k cstride <= npc
    for (int k = threadIdx.x; k < nc; k += kBlock) coarse[k] = cum[(long long)k * cstride];
    __syncthreads();
    const long long g = ((long long)blockIdx.x * kBlock + threadIdx.x) / kArcLanes;
    const int l = threadIdx.x & (kArcLanes - 1);
    if (g >= ns) return;   // whole lane groups leave together
    const int i = (int)g;
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

int arc_pieces(const DCurve& c) { return (c.n - c.p) * kArcSub; }

template <bool ADAPT>
static hipError_t launch_arclength_t(const DCurve& c, int ns, double lam, double* len, double* cum, double* su,
                                     int* ss, hipStream_t st)
{
    const int npc = arc_pieces(c), cs = arc_coarse_stride(npc);
    const dim3 gp((unsigned)(((long long)npc * 8 + kBlock - 1) / kBlock));
    const dim3 gs((unsigned)(((long long)ns * kArcLanes + kBlock - 1) / kBlock));
#define SWEEP_CASE(P)                                                                                           \
    case P:                                                                                                     \
        hipLaunchKernelGGL((k_arc_pieces<P, ADAPT>), gp, dim3(kBlock), 0, st, c, npc, lam, len);                \
        hipLaunchKernelGGL(k_arc_cumsum, dim3(1), dim3(kScanThreads), 0, st, len, npc, cum);                   \
        hipLaunchKernelGGL((k_arc_params<P, ADAPT>), gs, dim3(kBlock), 0, st, c, ns, npc, cs, lam, cum, su, ss); \
        break;
    switch (c.p) {
        SWEEP_CASE(1) SWEEP_CASE(2) SWEEP_CASE(3) SWEEP_CASE(4) SWEEP_CASE(5) SWEEP_CASE(6) SWEEP_CASE(7)
    default: return hipErrorInvalidValue;
    }
#undef SWEEP_CASE
    return hipGetLastError();
}

hipError_t launch_arclength(const DCurve& c, int ns, double lam, double* len, double* cum, double* su, int* ss,
                            hipStream_t st)
{
    return lam != 0.0 ? launch_arclength_t<true>(c, ns, lam, len, cum, su, ss, st)
                      : launch_arclength_t<false>(c, ns, lam, len, cum, su, ss, st);
}

// ------------------------------------------------------------ triangles

// The list is 6 ints per quad (i, j) in row-major quad order: triangles
// (i,j) (i,j+1) (i+1,j) and (i+1,j) (i,j+1) (i+1,j+1), j+1 modulo n_v for a
// closed profile; vertex (i, j) has index i n_v + j (below 2^31).
struct TriGrid {
    int n_v, nq;       // vertices and quads per row
    FastDiv dq;        // division by nq
};

struct Quad {
    int a, b;          // (i, j) and (i, j+1); the next row adds n_v
};

__device__ __forceinline__ Quad quad_of(const TriGrid& G, int i, int j)
{
    const int j1 = j + 1 < G.n_v ? j + 1 : 0;
    return Quad{i * G.n_v + j, i * G.n_v + j1};
}

// Int k (0..5) of a quad: a b c c b d.
__device__ __forceinline__ int quad_int(const TriGrid& G, const Quad& Q, int k)
{
    switch (k) {
    case 0: return Q.a;
    case 1: case 4: return Q.b;
    case 2: case 3: return Q.a + G.n_v;
    default: return Q.b + G.n_v;
    }
}

// kTriQuads quads per block (6 kTriQuads = 3072 ints = 3 x 256 x 16 bytes):
// thread t writes the 16-byte pieces t, t + 256 and t + 512 of its block's
// tile, so each store instruction of a wave covers 1 KiB of consecutive
// memory.  A piece starts at int 4c of the tile: quad (2c)/3 of it, at int
// 0, 2 or 4 of that quad, and runs into the next quad when it starts at 4.
// The tile's first quad (i0, j0) is divided out once; a piece's quad is
// then j0 + (2c)/3 quads along, at most kTriQuads past it (one more small
// division).  tri 16-byte aligned.
constexpr int kTriQuads = 512;

__global__ __launch_bounds__(kBlock) void k_triangles16(TriGrid G, long long n_quads, int* __restrict__ tri)
{
    typedef int i4 __attribute__((ext_vector_type(4)));
    const long long qb = (long long)blockIdx.x * kTriQuads;
    const int i0 = (int)(qb / G.nq), j0 = (int)(qb - (long long)i0 * G.nq);
    int* __restrict__ base = tri + 6 * qb;
    const int n_ints = (int)min((long long)kTriQuads, n_quads - qb) * 6;   // ints of this tile
    const int n = G.n_v;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int c = r * kBlock + threadIdx.x;
        const int e0 = 4 * c;
        if (e0 >= n_ints) break;
        const int ql = (2 * c) / 3, k0 = e0 - 6 * ql;
        const int jj = j0 + ql;
        const int di = fdiv((unsigned)jj, G.dq);
        const int i = i0 + di, j = jj - di * G.nq;
        // this quad: a = (i, j), b = (i, j+1 mod n_v); the next one: a2, b2
        const int a = i * n + j, b = j + 1 < n ? a + 1 : i * n;
        const bool next_row = j + 1 >= G.nq;
        const int a2 = next_row ? (i + 1) * n : a + 1;
        const int b2 = next_row ? a2 + 1 : (j + 2 < n ? a + 2 : i * n);
        // ints k0..k0+3 of the pattern a b c c b d | a2 b2 ..., c = a+n, d = b+n
        const bool z = k0 == 0, t2 = k0 == 2;
        const int v0 = z ? a : (t2 ? a + n : b);
        const int v1 = z ? b : (t2 ? a + n : b + n);
        const int v2 = z ? a + n : (t2 ? b : a2);
        const int v3 = z ? a + n : (t2 ? b + n : b2);
        if (e0 + 4 <= n_ints) {
            __builtin_nontemporal_store((i4){v0, v1, v2, v3}, reinterpret_cast<i4*>(base + e0));
        } else {
            const int v[4] = {v0, v1, v2, v3};
            for (int s = 0; e0 + s < n_ints; ++s) base[e0 + s] = v[s];
        }
    }
}

// Any alignment: one thread per int.
__global__ __launch_bounds__(kBlock) void k_triangles1(TriGrid G, long long n_ints, int* __restrict__ tri)
{
    const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n_ints) return;
    const unsigned q = (unsigned)(e / 6);
    const int i = fdiv(q, G.dq), j = (int)q - i * G.nq;
    tri[e] = quad_int(G, quad_of(G, i, j), (int)(e - 6LL * q));
}

hipError_t launch_triangles(int n_u, int n_v, int closed_v, int* tri, hipStream_t st)
{
    TriGrid G;
    G.n_v = n_v;
    G.nq = closed_v ? n_v : n_v - 1;
    unsigned long long m;
    int sh;
    fastdiv_constants(G.nq, &m, &sh);
    G.dq = FastDiv{m, sh, G.nq};
    const long long n_quads = (long long)(n_u - 1) * G.nq;   // below 2^31: the grid has fewer vertices
    if (n_quads == 0) return hipSuccess;
    if (((uintptr_t)tri & 15) == 0) {
        const long long grid = (n_quads + kTriQuads - 1) / kTriQuads;
        hipLaunchKernelGGL(k_triangles16, dim3((unsigned)grid), dim3(kBlock), 0, st, G, n_quads, tri);
    } else {
        const long long n_ints = 6 * n_quads;
        const long long grid = (n_ints + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_triangles1, dim3((unsigned)grid), dim3(kBlock), 0, st, G, n_ints, tri);
    }
    return hipGetLastError();
}

}  // namespace sweep

#pragma clang fp contract(fast)
