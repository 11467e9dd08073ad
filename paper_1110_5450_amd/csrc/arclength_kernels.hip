// arclength_kernels.hip -- arc-length sampling of the path (kernels over
// arclength.hpp) and the grid's triangle list.
#include "arclength.hpp"
#include "surface_common.hpp"

#pragma clang fp contract(off)

namespace sweep {

template <int P, bool ADAPT, bool RAT>
__global__ __launch_bounds__(kBlock) void k_arc_pieces(DCurve c, int nspan, double lam, double* __restrict__ len)
{
    __shared__ double setup[kWaves][SpanDeriv<P>::kDoubles];
    const int w = threadIdx.x >> 6;
    const long long si = (long long)blockIdx.x * kWaves + w;
    if (si >= nspan) return;   // whole waves leave together
    arc_span<P, ADAPT, RAT>(c, (int)si, threadIdx.x & 63, lam, setup[w], len);
}

__global__ __launch_bounds__(kScanThreads) void k_arc_cumsum(const double* __restrict__ len, int npc,
                                                             double* __restrict__ cum)
{
    arc_cumsum_block(len, npc, cum);
}

template <int P, bool ADAPT, bool RAT>
__global__ __launch_bounds__(kBlock) void k_arc_params(DCurve c, int ns, int npc, int cstride, double lam,
                                                       const double* __restrict__ cum, double* __restrict__ su,
                                                       int* __restrict__ ss)
{
    __shared__ double coarse[kArcCoarseMax];
    __shared__ double setup[kBlock / kArcLanes][SpanDeriv<P>::kDoubles];
    const int nc = npc / cstride + 1;   // coarse[k] = cum[k cstride], k cstride <= npc
    for (int k = threadIdx.x; k < nc; k += kBlock) coarse[k] = cum[(long long)k * cstride];
    __syncthreads();
    const long long g = ((long long)blockIdx.x * kBlock + threadIdx.x) / kArcLanes;
    if (g >= ns) return;   // whole lane groups leave together
    arc_param<P, ADAPT, RAT>(c, (int)g, threadIdx.x & (kArcLanes - 1), ns, npc, cstride, nc, lam, cum, coarse,
                             setup[threadIdx.x / kArcLanes], su, ss);
}

int arc_pieces(const DCurve& c) { return arc_piece_count(c.n, c.p); }

template <bool ADAPT, bool RAT>
static hipError_t launch_arclength_t(const DCurve& c, int ns, double lam, double* len, double* cum, double* su,
                                     int* ss, hipStream_t st)
{
    const int npc = arc_pieces(c), cs = arc_coarse_stride(npc), nspan = c.n - c.p;
    const dim3 gp((unsigned)((nspan + kWaves - 1) / kWaves));
    const dim3 gs((unsigned)(((long long)ns * kArcLanes + kBlock - 1) / kBlock));
#define SWEEP_CASE(P)                                                                                      \
    case P:                                                                                                \
        hipLaunchKernelGGL((k_arc_pieces<P, ADAPT, RAT>), gp, dim3(kBlock), 0, st, c, nspan, lam, len);      \
        hipLaunchKernelGGL(k_arc_cumsum, dim3(1), dim3(kScanThreads), 0, st, len, npc, cum);              \
        hipLaunchKernelGGL((k_arc_params<P, ADAPT, RAT>), gs, dim3(kBlock), 0, st, c, ns, npc, cs, lam, cum, su, \
                           ss);                                                                            \
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
    if (c.w) return lam != 0.0 ? launch_arclength_t<true, true>(c, ns, lam, len, cum, su, ss, st)
                               : launch_arclength_t<false, true>(c, ns, lam, len, cum, su, ss, st);
    return lam != 0.0 ? launch_arclength_t<true, false>(c, ns, lam, len, cum, su, ss, st)
                      : launch_arclength_t<false, false>(c, ns, lam, len, cum, su, ss, st);
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
