// backward_kernels.hip -- adjoint of the positions and normals with respect
// to the path and profile control points, for a batch.  With w = dL/dX and
// X_ij = x_i + S_x r_i + S_y s_i + S_z t_i:
//   dL/dx_i (direct)    = sum_j w_ij
//   dL/dr_i, ds_i, dt_i = sum_j S_{x,y,z}(v_j) w_ij
//   dL/dS_j             = sum_i R_i^T w_ij
// The frame is r_{i+1} = M_i r_i with M_i R_i = R_{i+1} (exact arithmetic),
// so the adjoint recurrence rbar_i = rbar_i^dir + M_i^T rbar_{i+1} becomes a
// suffix sum in frame coordinates: R_i^T rbar_i = sum_{k>=i} R_k^T rbar_k^dir.
// Each step M_i = H2 H1 is then differentiated through its two reflections
// (chord x_{i+1} - x_i and tangents t_i, t_{i+1}), t = C'/|C'| through the
// normalisation, r_0 through the initial-normal rule, and x, C' to the
// control points through the basis functions.  Every sum runs in FP64 in a
// fixed order: the result does not depend on scheduling.
//
// Normals (g = dL/dN, optional): N_ij = R_i n_ij with n = m/|m|,
// m = q_j x u_ij in frame coordinates, q = S' and
// u = (S_z a, S_z b, L - S_x a - S_y b), a = r.C''/L, b = s.C''/L, L = |C'|.
// With gh = R^T g, mb = (gh - (gh.n) n)/|m|, qb = u x mb, ub = mb x q:
//   dL/dr_i, ds_i, dt_i += sum_j n_{x,y,z} g_ij
//   dL/da_i = sum_j (ub_x S_z - ub_z S_x),  dL/db_i = sum_j (ub_y S_z - ub_z S_y),
//   dL/dL_i = sum_j ub_z
//   dL/dS_j += sum_i (-ub_z a, -ub_z b, ub_x a + ub_y b),  dL/dS'_j = sum_i qb
// and a, b, L pass on to r, s, C'' and C'.  Where |m| is 0 or not finite the
// normal is the constant 0 and passes nothing.
//
// kbw_reduce   one wave per (sweep, group of G rows, 64 columns): streaming
//              read of w through an LDS tile, per-row partials over the 64
//              columns and per-column partials over the G rows.
// kbw_rows, kbw_samples, kbw_final: the rest of the adjoint (described
//              with the kernels below).
#include "basis_ders.hpp"
#include "frame_common.hpp"

namespace sweep {

// One block per unit (sweep, kWaves groups of G rows, segment of 64
// columns), one wave per group; each wave's LDS tiles are its own (no block
// barriers until the end).  Lane = column j loads its G x 3 values of w
// (coalesced) and keeps them in registers for the column sums
//   h_j += R_i^T w_ij over the group's rows, added over the block's waves
//   in wave order at the end (one column partial per unit);
// the values also go to an LDS tile (rows padded to 65 elements: no bank
// conflicts) from which lane = (component c, row r, half h) forms the row
// sums over 32 of the 64 columns; the two halves are added in a fixed order
// (h = 0 first).  Small tiles keep five blocks per CU resident.
// With NRM the lane also loads g for its G rows and forms the normal terms:
// column sums in registers, row sums through the LDS tile.  grad may be null
// (no position term).
// The LDS tiles of kbw_reduce are private to a wave: ordering its own LDS
// accesses needs no block barrier.  LDS operations of one wave execute in
// order; the wave-scope fences keep the compiler from moving them across
// this point.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T, bool NRM>
__global__ __launch_bounds__(kBlock) void kbw_reduce(const BatchDesc* __restrict__ descs,
                                                     const int4* __restrict__ units, int n_units,
                                                     const T* __restrict__ grad, const T* __restrict__ gnrm,
                                                     const double* __restrict__ rows,
                                                     const double* __restrict__ ptab, double* __restrict__ rowpart,
                                                     double* __restrict__ colpart)
{
    constexpr int G = bw_row_group<T>();
    constexpr int RP = NRM ? kRowPartNrm : kRowPart;
    constexpr int CP = NRM ? kColPartNrm : kColPart;
    __shared__ T lw[kWaves][3][G][65];
    __shared__ double ls[kWaves][3][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int unit = blockIdx.x;
    const bool live = unit < n_units;   // block-uniform
    int4 un = make_int4(0, 0, 0, 0);
    if (live) un = units[unit];
    const BatchDesc& d = descs[un.x];
    const int n_u = d.n_u, n_v = d.n_v;
    const int g = un.y * kWaves + wave, seg = un.z;   // this wave's group of G rows
    const int j = seg * 64 + lane;
    const bool vj = live && j < n_v;
    {
        double S0 = 0.0, S1 = 0.0, S2 = 0.0;
        if (vj) {
            const double* q = ptab + 8 * (d.ptab_off + j);
            S0 = q[0]; S1 = q[1]; S2 = q[2];
        }
        ls[wave][0][lane] = S0; ls[wave][1][lane] = S1; ls[wave][2][lane] = S2;
    }
    // column sums over this wave's G rows
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;
    V3<double> hD = mk(0.0, 0.0, 0.0);
    const int i0 = g * G;
    if (live && i0 < n_u) {   // wave-uniform
    const int nr = min(G, n_u - i0);
    wave_lds_sync();   // the previous group's LDS tiles are consumed
    T w[3][G];
    {
        const size_t P = (size_t)d.plane;   // plane stride of the batched layout
        const T* w0 = grad ? grad + d.out_off : nullptr;
#pragma unroll
        for (int r = 0; r < G; ++r) {
            w[0][r] = w[1][r] = w[2][r] = T(0);
            if (w0 && vj && r < nr) {
                const size_t v = (size_t)(i0 + r) * (size_t)n_v + (size_t)j;
                w[0][r] = __builtin_nontemporal_load(w0 + v);
                w[1][r] = __builtin_nontemporal_load(w0 + P + v);
                w[2][r] = __builtin_nontemporal_load(w0 + 2 * P + v);
            }
        }
#pragma unroll
        for (int r = 0; r < G; ++r) {
            lw[wave][0][r][lane] = w[0][r]; lw[wave][1][r][lane] = w[1][r]; lw[wave][2][r][lane] = w[2][r];
        }
    }
    const double* R0 = rows + 16 * (d.row_off + i0);
    if (vj) {
#pragma unroll
        for (int r = 0; r < G; ++r) {
            if (r < nr) {
                const double* R = R0 + 16 * r;
                const double a = (double)w[0][r], b = (double)w[1][r], c = (double)w[2][r];
                h0 += R[3] * a + R[4] * b + R[5] * c;
                h1 += R[6] * a + R[7] * b + R[8] * c;
                h2 += R[9] * a + R[10] * b + R[11] * c;
            }
        }
    }
    wave_lds_sync();
    // lane = ((c * G + r) << 1) | h
    const int h = lane & 1, cr = lane >> 1, r = cr % G, c = cr / G;
    const bool act = live && c < 3 && r < nr;
    double a0 = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    if (act) {
        const int ncol = min(64, n_v - seg * 64);
        const int j0 = h * 32, j1 = min(ncol, j0 + 32);
        for (int jj = j0; jj < j1; ++jj) {
            const double v = (double)lw[wave][c][r][jj];
            a0 += v;
            ax += ls[wave][0][jj] * v;
            ay += ls[wave][1][jj] * v;
            az += ls[wave][2][jj] * v;
        }
    }
    // the second half's sums from the neighbouring lane (every lane takes part)
    const double b0 = __shfl_xor(a0, 1, 64), bx = __shfl_xor(ax, 1, 64);
    const double by = __shfl_xor(ay, 1, 64), bz = __shfl_xor(az, 1, 64);
    if (act && h == 0) {
        double* q = rowpart + RP * (d.rowpart_off + (size_t)seg * n_u + i0 + r);
        q[c] = a0 + b0; q[3 + c] = ax + bx; q[6 + c] = ay + by; q[9 + c] = az + bz;
    }
    if (NRM) {
        // The normal terms.  Row sums go through the wave's (now free) LDS
        // tile: lanes write their 12 values of a row, then lane (e, k),
        // e < 12, k < 4, sums value e over columns 16k .. 16k+15 and the four
        // parts are added in a fixed order.
        V3<double> S = mk(0.0, 0.0, 0.0), q = S;
        if (vj) {
            const double* pq = ptab + 8 * (d.ptab_off + j);
            S = mk(pq[0], pq[1], pq[2]);
            q = mk(pq[3], pq[4], pq[5]);
        }
        const size_t P = (size_t)d.plane;
        const T* g0 = gnrm + d.out_off;
        double* buf = reinterpret_cast<double*>(&lw[wave][0][0][0]);   // 12 x 65 doubles
        static_assert(sizeof(lw[0]) >= 12 * 65 * sizeof(double), "LDS tile too small for the normal terms");
        const int e = lane >> 2, kq = lane & 3;
        for (int r = 0; r < G; ++r) {
            double cv[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) cv[k] = 0.0;
            if (vj && r < nr) {
                const double* R = R0 + 16 * r;
                const size_t v = (size_t)(i0 + r) * (size_t)n_v + (size_t)j;
                const V3<double> gv = mk((double)__builtin_nontemporal_load(g0 + v),
                                         (double)__builtin_nontemporal_load(g0 + P + v),
                                         (double)__builtin_nontemporal_load(g0 + 2 * P + v));
                const V3<double> rr = mk(R[3], R[4], R[5]), ss = mk(R[6], R[7], R[8]), tt = mk(R[9], R[10], R[11]);
                const double L = R[12], a = R[13], b = R[14];
                const V3<double> u = mk(S.z * a, S.z * b, L - S.x * a - S.y * b);
                const V3<double> m = cross(q, u);
                const double mm = dot(m, m);
                if (mm > 0.0 && mm < INFINITY) {
                    const double inv = 1.0 / sqrt(mm);
                    const V3<double> n = inv * m;
                    const V3<double> gh = mk(dot(rr, gv), dot(ss, gv), dot(tt, gv));
                    const V3<double> mb = inv * (gh - dot(gh, n) * n);
                    const V3<double> qb = cross(u, mb), ub = cross(mb, q);
                    cv[0] = n.x * gv.x; cv[1] = n.x * gv.y; cv[2] = n.x * gv.z;
                    cv[3] = n.y * gv.x; cv[4] = n.y * gv.y; cv[5] = n.y * gv.z;
                    cv[6] = n.z * gv.x; cv[7] = n.z * gv.y; cv[8] = n.z * gv.z;
                    cv[9] = ub.x * S.z - ub.z * S.x;
                    cv[10] = ub.y * S.z - ub.z * S.y;
                    cv[11] = ub.z;
                    h0 -= ub.z * a;
                    h1 -= ub.z * b;
                    h2 += ub.x * a + ub.y * b;
                    hD = hD + qb;
                }
            }
            wave_lds_sync();   // the tile's previous contents are consumed
#pragma unroll
            for (int k = 0; k < 12; ++k) buf[65 * k + lane] = cv[k];
            wave_lds_sync();
            double part = 0.0;
            if (lane < 48)
                for (int jj = 16 * kq; jj < 16 * kq + 16; ++jj) part += buf[65 * e + jj];
            part += __shfl_xor(part, 1, 64);
            part += __shfl_xor(part, 2, 64);
            if (live && r < nr && lane < 48 && kq == 0)
                rowpart[RP * (d.rowpart_off + (size_t)seg * n_u + i0 + r) + kRowPart + e] = part;
        }
    }
    }   // the wave's rows
    // the unit's column partial: the waves' sums added in wave order,
    // through the (now free) LDS tiles
    __syncthreads();
    double* hc = reinterpret_cast<double*>(&lw[0][0][0][0]);   // kWaves x CP x 64
    static_assert(sizeof(lw) >= sizeof(double) * kWaves * kColPartNrm * 64, "LDS tile too small for the column sums");
    hc[(wave * CP + 0) * 64 + lane] = h0;
    hc[(wave * CP + 1) * 64 + lane] = h1;
    hc[(wave * CP + 2) * 64 + lane] = h2;
    if (NRM) {
        hc[(wave * CP + 3) * 64 + lane] = hD.x;
        hc[(wave * CP + 4) * 64 + lane] = hD.y;
        hc[(wave * CP + 5) * 64 + lane] = hD.z;
    }
    __syncthreads();
    if (wave == 0 && vj) {
        double* q = colpart + CP * (d.colpart_off + (size_t)un.y * n_v + j);
#pragma unroll
        for (int e = 0; e < CP; ++e) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += hc[(w * CP + e) * 64 + lane];
            q[e] = t;
        }
    }
}

// Basis values N_{s-P+j,P}(u) and first derivatives, j = 0..P, and (d2N
// not null) second derivatives.
template <int P>
__device__ __forceinline__ void basis_vals(const DCurve& c, double u, int s, double* N, double* dN, double* d2N)
{
    double Uk[2 * P + 1];
#pragma unroll
    for (int m = 0; m < 2 * P; ++m) Uk[m] = knot(c, s - P + 1 + m);
    double B[P + 1];
    double D1[P > 0 ? P : 1];
    double D2[P > 1 ? P - 1 : 1];
    B[0] = 1.0;
    if (P - 1 == 0) D1[0] = 1.0;
    if (P - 2 == 0) D2[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= P; ++q) {
        double nb_[P + 1];
        double carry = 0.0;
#pragma unroll
        for (int j = 0; j < q; ++j) {
            const double lo = Uk[P - q + j], hi = Uk[P + j];
            const double tmp = B[j] / (hi - lo);
            nb_[j] = carry + (hi - u) * tmp;
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
    }
    // C' = sum_j D1[j] Q_j with Q_j = P (P_{j+1} - P_j) / (U_{s+j+1} - U_{s-P+j+1})
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        double v = 0.0;
        if (j >= 1) v += D1[j - 1] / (Uk[P + j - 1] - Uk[j - 1]);
        if (j < P) v -= D1[j] / (Uk[P + j] - Uk[j]);
        N[j] = B[j];
        dN[j] = (double)P * v;
    }
    if (d2N) {
        // first derivatives of the degree P-1 functions N_{s-P+1+j,P-1}
        // from the degree P-2 values, then the same difference rule again
        double E1[P > 0 ? P : 1];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            double v = 0.0;
            if (P >= 2) {
                if (j >= 1) v += D2[j - 1] / (Uk[P - 1 + j] - Uk[j]);
                if (j <= P - 2) v -= D2[j] / (Uk[P + j] - Uk[j + 1]);
            }
            E1[j] = (double)(P - 1) * v;
        }
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            double v = 0.0;
            if (j >= 1) v += E1[j - 1] / (Uk[P + j - 1] - Uk[j - 1]);
            if (j < P) v -= E1[j] / (Uk[P + j] - Uk[j]);
            d2N[j] = (double)P * v;
        }
    }
}

// Basis of sample i of ns (any degree up to kMaxDeg): span and values, and
// (d2N not null) second derivatives.  For a rational curve the values are
// those of the rational basis R_k = w_k N_k / W, R_k' = w_k (N_k' W - N_k W')
// / W^2 and R_k'' = w_k (N_k''/W - 2 N_k' W'/W^2 - N_k W''/W^2
// + 2 N_k W'^2/W^3) (W = sum w_k N_k): the derivatives of C, C' and C'' with
// respect to control point k.
__device__ __forceinline__ int sample_basis(const DCurve& c, int i, int ns, double* N, double* dN,
                                            double* d2N = nullptr)
{
    const double u = sample_param(c, i, ns);
    const int s = sample_span(c, i, ns, u);
    switch (c.p) {
    case 1: basis_vals<1>(c, u, s, N, dN, d2N); break;
    case 2: basis_vals<2>(c, u, s, N, dN, d2N); break;
    case 3: basis_vals<3>(c, u, s, N, dN, d2N); break;
    case 4: basis_vals<4>(c, u, s, N, dN, d2N); break;
    case 5: basis_vals<5>(c, u, s, N, dN, d2N); break;
    case 6: basis_vals<6>(c, u, s, N, dN, d2N); break;
    default: basis_vals<7>(c, u, s, N, dN, d2N); break;
    }
    if (c.w) {
        double W = 0.0, W1 = 0.0, W2 = 0.0;
        for (int j = 0; j <= c.p; ++j) {
            const double wk = weight_at(c, s - c.p + j);
            W += wk * N[j];
            W1 += wk * dN[j];
            if (d2N) W2 += wk * d2N[j];
        }
        for (int j = 0; j <= c.p; ++j) {
            const double wk = weight_at(c, s - c.p + j);
            const double Rj = wk * N[j] / W;
            if (d2N)
                d2N[j] = wk * (d2N[j] / W - 2.0 * dN[j] * W1 / (W * W) - N[j] * W2 / (W * W) +
                               2.0 * N[j] * W1 * W1 / (W * W * W));
            dN[j] = wk * (dN[j] * W - N[j] * W1) / (W * W);
            N[j] = Rj;
        }
    }
    return s;
}

// Adjoint of H(v) w = w - (2 (v.w)/(v.v)) v with respect to v, given the
// adjoint zb of H(v) w.
__device__ __forceinline__ V3<double> reflect_adj(V3<double> v, V3<double> w, V3<double> zb)
{
    const double c = dot(v, v), vw = dot(v, w), vz = dot(v, zb);
    return (-2.0 / c) * (vz * w + vw * zb) + (4.0 * vw * vz / (c * c)) * v;
}

struct StepAdj {
    V3<double> x0, x1, t0, t1;   // contributions to samples i and i+1
};

// Adjoint of r_{i+1} = H2 H1 r_i with respect to (x_i, x_{i+1}, t_i, t_{i+1}),
// given yb = dL/dr_{i+1}.  A tangent-reversal step (|v2|^2 <= 1e-24) is
// treated as locally constant.
__device__ __forceinline__ StepAdj step_adjoint(V3<double> xa, V3<double> xb, V3<double> ta, V3<double> tb,
                                                V3<double> ra, V3<double> yb)
{
    StepAdj o;
    const V3<double> z = mk(0.0, 0.0, 0.0);
    o.x0 = z; o.x1 = z; o.t0 = z; o.t1 = z;
    V3<double> v1 = xb - xa;
    double c1 = dot(v1, v1);
    const bool zero_chord = c1 == 0.0;
    if (zero_chord) { v1 = ta; c1 = dot(v1, v1); }
    const double b1 = 2.0 / c1;
    const V3<double> rL = ra - (b1 * dot(v1, ra)) * v1;
    const V3<double> tL = ta - (b1 * dot(v1, ta)) * v1;
    const V3<double> v2 = tb - tL;
    const double c2 = dot(v2, v2);
    if (!(c2 > 1e-24)) return o;
    const double b2 = 2.0 / c2;
    const V3<double> v2b = reflect_adj(v2, rL, yb);
    const V3<double> y1b = yb - (b2 * dot(v2, yb)) * v2;
    V3<double> v1b = reflect_adj(v1, ra, y1b);
    const V3<double> tLb = mk(-v2b.x, -v2b.y, -v2b.z);
    o.t1 = v2b;
    o.t0 = tLb - (b1 * dot(v1, tLb)) * v1;
    v1b = v1b + reflect_adj(v1, ta, tLb);
    if (zero_chord) o.t0 = o.t0 + v1b;
    else { o.x1 = v1b; o.x0 = mk(-v1b.x, -v1b.y, -v1b.z); }
    return o;
}

// Threads per output in the adjoint's gathers.
constexpr int kMaxParts = 8;

// First index in the non-decreasing v[0..n) with v[index] >= key (n if none).
__device__ __forceinline__ int lower_bound_int(const int* v, int n, int key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (v[m] >= key) hi = m; else lo = m + 1;
    }
    return lo;
}

struct RowRec {
    V3<double> x, r, s, t;
    double L;
};
__device__ __forceinline__ RowRec row_at(const double* R)
{
    return RowRec{mk(R[0], R[1], R[2]), mk(R[3], R[4], R[5]), mk(R[6], R[7], R[8]), mk(R[9], R[10], R[11]), R[12]};
}

// Inclusive suffix sum of 3-vectors over the block (thread 255 first); block
// total in `total`.  Fixed combination order.
__device__ V3<double> block_suffix_sum(V3<double> v, double (*lds)[3], V3<double>& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double ox = __shfl_down(v.x, d, 64), oy = __shfl_down(v.y, d, 64), oz = __shfl_down(v.z, d, 64);
        if (lane + d < 64) v = v + mk(ox, oy, oz);
    }
    if (lane == 0) { lds[w][0] = v.x; lds[w][1] = v.y; lds[w][2] = v.z; }
    __syncthreads();
    V3<double> later = mk(0.0, 0.0, 0.0), tot = later;
    for (int k = kWaves - 1; k >= 0; --k) {
        const V3<double> a = mk(lds[k][0], lds[k][1], lds[k][2]);
        if (k > w) later = later + a;
        tot = tot + a;
    }
    total = tot;
    __syncthreads();
    return v + later;
}

// Row records of the partial sums: kRowPart = 12 values for the positions
// (sum w, dL/dr, dL/ds, dL/dt), kRowPartNrm = 24 with the normal terms
// (then sum n_x g, sum n_y g, sum n_z g, dL/da, dL/db, dL/dL); column records
// hold dL/dS (kColPart = 3), and dL/dS' after it with the normal terms
// (kColPartNrm = 6).

// The normal terms' share of dL/dr_i, dL/ds_i and dL/dt_i: sum_j n_{x,y,z} g_ij
// and, through a = r.C''/L and b = s.C''/L, (dL/da) C''/L and (dL/db) C''/L
// (C'' from the second-derivative basis).  Written over the record's
// direct terms (values 3..11), which then hold the totals.
__device__ __forceinline__ void fold_normal_frame_terms(const DCurve& path, int i, int n_u, const RowRec& R,
                                                        double* a)
{
    V3<double> Gr = mk(a[3], a[4], a[5]) + mk(a[12], a[13], a[14]);
    V3<double> Gs = mk(a[6], a[7], a[8]) + mk(a[15], a[16], a[17]);
    const V3<double> Gt = mk(a[9], a[10], a[11]) + mk(a[18], a[19], a[20]);
    if (R.L > 0.0) {
        double Nv[kMaxDeg + 1], dN[kMaxDeg + 1], d2N[kMaxDeg + 1];
        const int s = sample_basis(path, i, n_u, Nv, dN, d2N);
        V3<double> C2 = mk(0.0, 0.0, 0.0);
        for (int j = 0; j <= path.p; ++j) C2 = C2 + d2N[j] * ctrl_pt(path, s - path.p + j);
        Gr = Gr + (a[21] / R.L) * C2;
        Gs = Gs + (a[22] / R.L) * C2;
    }
    a[3] = Gr.x; a[4] = Gr.y; a[5] = Gr.z;
    a[6] = Gs.x; a[7] = Gs.y; a[8] = Gs.z;
    a[9] = Gt.x; a[10] = Gt.y; a[11] = Gt.z;
}

// The adjoint after kbw_reduce, in three launches:
//
// kbw_rows     one block per (sweep, chunk of kBlock u-samples): finishes the
//              row sums (fixed order over the column segments), folds in the
//              normal terms' share of dL/dr, dL/ds, dL/dt, forms each row's
//              direct term d_i = R_i^T rbar_i^dir and its suffix sum inside
//              the chunk; the chunk's total goes to ctot.
// kbw_samples  one block per (sweep, chunk): rho_i = (suffix inside the
//              chunk) + (totals of the later chunks, added from the last one
//              down), then the per-sample adjoint of x_i and C'_i (step
//              adjoints, the initial-normal rule at i = 0, the tangent
//              normalisation) and its basis contributions to the control
//              points of the sample's span.
// kbw_final    one block per sweep: finishes the column sums, the profile
//              samples' basis contributions and the gathers per control point.
// Sums run in FP64 in a fixed order: the result does not depend on
// scheduling.

__device__ __forceinline__ DCurve path_curve(const BatchDesc& d, const double* path_ctrl, const double* path_w,
                                             const double* knots)
{
    return DCurve{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr,
                  d.n_path, d.p_path, 0, d.n_path, path_w ? path_w + d.path_ctrl_off : nullptr};
}
__device__ __forceinline__ DCurve prof_curve(const BatchDesc& d, const double* prof_ctrl, const double* prof_w,
                                             const double* knots)
{
    return DCurve{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr,
                  d.n_prof, d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof,
                  prof_w ? prof_w + d.prof_ctrl_off : nullptr};
}

// Chunk totals of the rows' direct terms: 3 doubles per (sweep, chunk), the
// chunks of sweep k starting at ctot_off(k) = sum of earlier chunk counts.
__global__ __launch_bounds__(kBlock) void kbw_rows(const BatchDesc* __restrict__ descs,
                                                   const int2* __restrict__ chunks,
                                                   const double* __restrict__ path_ctrl,
                                                   const double* __restrict__ path_w,
                                                   const double* __restrict__ knots,
                                                   const double* __restrict__ rows, const double* rowpart,
                                                   double* rowacc, double* sfx, double* ctot, int nrm)
{
    __shared__ double lds3[kWaves][3];
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const DCurve path = path_curve(d, path_ctrl, path_w, knots);
    const int rp = nrm ? kRowPartNrm : kRowPart;
    const int n_u = d.n_u;
    const int i = ch.y * kBlock + threadIdx.x;
    V3<double> di = mk(0.0, 0.0, 0.0);
    if (i < n_u) {
        double a[kRowPartNrm];
#pragma unroll
        for (int e = 0; e < kRowPartNrm; ++e) a[e] = 0.0;
        for (int sgi = 0; sgi < d.nseg; ++sgi) {
            const double* q = rowpart + rp * (d.rowpart_off + (size_t)sgi * n_u + i);
#pragma unroll
            for (int e = 0; e < kRowPartNrm; ++e)
                if (e < rp) a[e] += q[e];
        }
        const RowRec R = row_at(rows + 16 * (d.row_off + (size_t)i));
        if (nrm) fold_normal_frame_terms(path, i, n_u, R, a);
        double* ra = rowacc + rp * (d.row_off + (size_t)i);
#pragma unroll
        for (int e = 0; e < kRowPartNrm; ++e)
            if (e < rp) ra[e] = a[e];
        const V3<double> Gr = mk(a[3], a[4], a[5]), Gs = mk(a[6], a[7], a[8]);
        const V3<double> rb = Gr + cross(Gs, R.t);
        di = mk(dot(R.r, rb), dot(R.s, rb), dot(R.t, rb));
    }
    V3<double> total;
    const V3<double> s = block_suffix_sum(di, lds3, total);
    if (i < n_u) {
        double* q = sfx + 3 * (d.row_off + (size_t)i);
        q[0] = s.x; q[1] = s.y; q[2] = s.z;
    }
    if (threadIdx.x == 0) {
        double* q = ctot + 3 * (d.ctot_off + ch.y);
        q[0] = total.x; q[1] = total.y; q[2] = total.z;
    }
}

// Totals of the sweep's chunks after chunk c, added from the last one down.
__device__ __forceinline__ V3<double> later_chunks(const double* ctot, const BatchDesc& d, int c)
{
    const int nc = (d.n_u + kBlock - 1) / kBlock;
    V3<double> carry = mk(0.0, 0.0, 0.0);
    for (int b = nc - 1; b > c; --b) {
        const double* q = ctot + 3 * (d.ctot_off + b);
        carry = carry + mk(q[0], q[1], q[2]);
    }
    return carry;
}

__global__ __launch_bounds__(kBlock) void kbw_samples(const BatchDesc* __restrict__ descs,
                                                      const int2* __restrict__ chunks,
                                                      const double* __restrict__ path_ctrl,
                                                      const double* __restrict__ path_w,
                                                      const double* __restrict__ knots, InitialNormal n0,
                                                      const double* __restrict__ rows, const double* rowacc,
                                                      const double* sfx, const double* ctot, double* sgrad,
                                                      int* spans_u, int nrm, double* xstash)
{
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const DCurve path = path_curve(d, path_ctrl, path_w, knots);
    const int rp = nrm ? kRowPartNrm : kRowPart;
    const int n_u = d.n_u;
    const int i = ch.y * kBlock + threadIdx.x;
    if (i >= n_u) return;
    const double* rows_k = rows + 16 * d.row_off;
    const V3<double> carry = later_chunks(ctot, d, ch.y);
    // rho of the next sample: the next chunk's suffix plus its own carry
    const bool next_in_chunk = threadIdx.x + 1 < kBlock;
    const V3<double> carry_next = next_in_chunk ? carry : later_chunks(ctot, d, ch.y + 1);
    auto rho_at = [&](int k, V3<double> c) {
        const double* q = sfx + 3 * (d.row_off + (size_t)k);
        return mk(q[0], q[1], q[2]) + c;
    };
    const RowRec R = row_at(rows_k + 16 * (size_t)i);
    // (with the normal terms, values 3..11 hold the totals: kbw_rows)
    const double* a = rowacc + rp * (d.row_off + (size_t)i);
    const V3<double> g = mk(a[0], a[1], a[2]), Gs = mk(a[6], a[7], a[8]), Gt = mk(a[9], a[10], a[11]);
    double Nv[kMaxDeg + 1], dN[kMaxDeg + 1], d2N[kMaxDeg + 1];
    const int s = sample_basis(path, i, n_u, Nv, dN, nrm ? d2N : nullptr);
    V3<double> C2b = mk(0.0, 0.0, 0.0);   // dL/dC'' (normal terms)
    double Lb = 0.0;                       // dL/dL, L = |C'| (normal terms)
    if (nrm) {
        if (R.L > 0.0) {
            const double* rr = rows_k + 16 * (size_t)i;
            C2b = divs(a[21] * R.r + a[22] * R.s, R.L);
            Lb = a[23] - (a[21] * rr[13] + a[22] * rr[14]) / R.L;
        }
    }
    V3<double> xb = g;
    V3<double> tb = Gt + cross(R.r, Gs);
    const V3<double> rh = rho_at(i, carry);
    const V3<double> rbar_i = rh.x * R.r + rh.y * R.s + rh.z * R.t;
    if (i + 1 < n_u) {
        const RowRec Rn = row_at(rows_k + 16 * (size_t)(i + 1));
        const V3<double> rn = rho_at(i + 1, carry_next);
        const V3<double> yb = rn.x * Rn.r + rn.y * Rn.s + rn.z * Rn.t;
        const StepAdj sa = step_adjoint(R.x, Rn.x, R.t, Rn.t, R.r, yb);
        xb = xb + sa.x0;
        tb = tb + sa.t0;
    }
    if (i >= 1) {
        const RowRec Rp = row_at(rows_k + 16 * (size_t)(i - 1));
        const StepAdj sa = step_adjoint(Rp.x, R.x, Rp.t, R.t, Rp.r, rbar_i);
        xb = xb + sa.x1;
        tb = tb + sa.t1;
    }
    if (i == 0) {
        // r_0 = q/|q|, q = e - (e.t_0) t_0 with e the initial normal or e_a
        V3<double> e;
        bool user = false;
        if (n0.enabled) {
            const V3<double> nn = mk(n0.v[0], n0.v[1], n0.v[2]);
            const V3<double> q = nn - dot(nn, R.t) * R.t;
            if (sqrt(dot(q, q)) > 1e-8) { e = nn; user = true; }
        }
        if (!user) {
            const double ax = fabs(R.t.x), ay = fabs(R.t.y), az = fabs(R.t.z);
            int k = 0;
            double best = ax;
            if (ay < best) { k = 1; best = ay; }
            if (az < best) k = 2;
            e = mk(k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0);
        }
        const double et = dot(e, R.t);
        const V3<double> q = e - et * R.t;
        const double ql = sqrt(dot(q, q));
        const V3<double> qb = divs(rbar_i - dot(R.r, rbar_i) * R.r, ql);
        tb = tb - (et * qb + dot(qb, R.t) * e);
    }
    // t = C'/|C'|; samples with C' = 0 carry a tangent and pass no gradient
    V3<double> cb = mk(0.0, 0.0, 0.0);
    if (R.L > 0.0) cb = divs(tb - dot(R.t, tb) * R.t, R.L) + Lb * R.t;
    spans_u[d.row_off + i] = s;
    if (xstash) {
        // dL/dC, dL/dC', dL/dC'' of the sample, for the knot and weight gradients
        double* q = xstash + 9 * (d.row_off + (size_t)i);
        q[0] = xb.x; q[1] = xb.y; q[2] = xb.z;
        q[3] = cb.x; q[4] = cb.y; q[5] = cb.z;
        q[6] = C2b.x; q[7] = C2b.y; q[8] = C2b.z;
    }
    double* sg = sgrad + 24 * (d.row_off + (size_t)i);
    for (int j = 0; j <= path.p; ++j) {
        V3<double> c = Nv[j] * xb + dN[j] * cb;
        if (nrm) c = c + d2N[j] * C2b;
        sg[3 * j] = c.x; sg[3 * j + 1] = c.y; sg[3 * j + 2] = c.z;
    }
}

__global__ __launch_bounds__(kBlock) void kbw_final(const BatchDesc* __restrict__ descs,
                                                    const double* __restrict__ path_ctrl,
                                                    const double* __restrict__ prof_ctrl,
                                                    const double* __restrict__ path_w,
                                                    const double* __restrict__ prof_w,
                                                    const double* __restrict__ knots, const double* colpart,
                                                    double* colacc, const double* sgrad, const int* spans_u,
                                                    double* qgrad, int* spans_v, double* __restrict__ gP,
                                                    double* __restrict__ gQ, int nrm)
{
    const int cp = nrm ? kColPartNrm : kColPart;
    __shared__ double lpart[kBlock][kColPartNrm];
    const BatchDesc d = descs[blockIdx.x];
    const DCurve path = path_curve(d, path_ctrl, path_w, knots);
    const DCurve prof = prof_curve(d, prof_ctrl, prof_w, knots);
    const int n_u = d.n_u, n_v = d.n_v;
    double* cacc = colacc + (size_t)cp * d.ptab_off;
    const double* sg = sgrad + 24 * d.row_off;
    const int* su = spans_u + d.row_off;
    double* qg = qgrad + 24 * d.ptab_off;
    int* sv = spans_v + d.ptab_off;

    // 1. column sums over the row groups
    {
        // column sums over the row groups: `parts` threads per column, each
        // over a contiguous range of groups, combined in part order
        const int parts = n_v <= kBlock ? min(kMaxParts, kBlock / n_v) : 1;
        for (int t = threadIdx.x; t < n_v * parts; t += kBlock) {
            const int j = t / parts, part = t % parts;
            const int g0 = (int)((long long)d.ngroup * part / parts);
            const int g1 = (int)((long long)d.ngroup * (part + 1) / parts);
            double h[kColPartNrm];
#pragma unroll
            for (int e = 0; e < kColPartNrm; ++e) h[e] = 0.0;
            for (int g = g0; g < g1; ++g) {
                const double* q = colpart + cp * (d.colpart_off + (size_t)g * n_v + j);
#pragma unroll
                for (int e = 0; e < kColPartNrm; ++e)
                    if (e < cp) h[e] += q[e];
            }
            if (parts == 1) {
#pragma unroll
                for (int e = 0; e < kColPartNrm; ++e)
                    if (e < cp) cacc[cp * (size_t)j + e] = h[e];
            } else {
#pragma unroll
                for (int e = 0; e < kColPartNrm; ++e) lpart[t][e] = h[e];
            }
        }
        __syncthreads();
        if (parts > 1)
            for (int j = threadIdx.x; j < n_v; j += kBlock) {
                double h[kColPartNrm];
#pragma unroll
                for (int e = 0; e < kColPartNrm; ++e) h[e] = 0.0;
                for (int part = 0; part < parts; ++part)
#pragma unroll
                    for (int e = 0; e < kColPartNrm; ++e) h[e] += lpart[j * parts + part][e];
#pragma unroll
                for (int e = 0; e < kColPartNrm; ++e)
                    if (e < cp) cacc[cp * (size_t)j + e] = h[e];
            }
    }

    __syncthreads();

    // profile samples: dL/dS_j = h_j to the profile basis
    for (int j = threadIdx.x; j < n_v; j += kBlock) {
        double Nv[kMaxDeg + 1], dN[kMaxDeg + 1];
        const int s = sample_basis(prof, j, n_v, Nv, dN);
        sv[j] = s;
        const double* ca = cacc + cp * (size_t)j;
        const V3<double> h = mk(ca[0], ca[1], ca[2]);
        const V3<double> hd = nrm ? mk(ca[3], ca[4], ca[5]) : mk(0.0, 0.0, 0.0);
        for (int l = 0; l <= prof.p; ++l) {
            const V3<double> c = Nv[l] * h + dN[l] * hd;
            double* q = qg + 24 * (size_t)j + 3 * l;
            q[0] = c.x; q[1] = c.y; q[2] = c.z;
        }
    }
    __threadfence_block();
    __syncthreads();

    // 4. gathers per control point over the samples whose span covers it
    //    (spans are non-decreasing in the sample index, so these samples are
    //    a contiguous range); `parts` threads per control point each sum a
    //    contiguous piece, combined in part order
    {
        const int parts = d.n_path <= kBlock ? min(kMaxParts, kBlock / d.n_path) : 1;
        for (int t = threadIdx.x; t < d.n_path * parts; t += kBlock) {
            const int k = t / parts, part = t % parts;
            const int lo = lower_bound_int(su, n_u, k);              // first span >= k
            const int hi = lower_bound_int(su, n_u, k + path.p + 1);  // first span - p > k
            const int a = lo + (int)((long long)(hi - lo) * part / parts);
            const int b = lo + (int)((long long)(hi - lo) * (part + 1) / parts);
            V3<double> acc = mk(0.0, 0.0, 0.0);
            for (int i = a; i < b; ++i) {
                const double* q = sg + 24 * (size_t)i + 3 * (k - (su[i] - path.p));
                acc = acc + mk(q[0], q[1], q[2]);
            }
            if (parts == 1) {
                double* o = gP + 3 * (d.path_ctrl_off + k);
                o[0] = acc.x; o[1] = acc.y; o[2] = acc.z;
            } else {
                lpart[t][0] = acc.x; lpart[t][1] = acc.y; lpart[t][2] = acc.z;
            }
        }
        __syncthreads();
        if (parts > 1)
            for (int k = threadIdx.x; k < d.n_path; k += kBlock) {
                V3<double> acc = mk(0.0, 0.0, 0.0);
                for (int part = 0; part < parts; ++part)
                    acc = acc + mk(lpart[k * parts + part][0], lpart[k * parts + part][1], lpart[k * parts + part][2]);
                double* o = gP + 3 * (d.path_ctrl_off + k);
                o[0] = acc.x; o[1] = acc.y; o[2] = acc.z;
            }
        __syncthreads();
    }
    {
        // basis indices wrapping onto control point l: l, and l + m, ... on
        // a closed curve
        const int parts = d.n_prof <= kBlock ? min(kMaxParts, kBlock / d.n_prof) : 1;
        for (int t = threadIdx.x; t < d.n_prof * parts; t += kBlock) {
            const int l = t / parts, part = t % parts;
            V3<double> acc = mk(0.0, 0.0, 0.0);
            for (int kk = l; kk < prof.nb; kk += d.n_prof) {
                const int lo = lower_bound_int(sv, n_v, kk);
                const int hi = lower_bound_int(sv, n_v, kk + prof.p + 1);
                const int a = lo + (int)((long long)(hi - lo) * part / parts);
                const int b = lo + (int)((long long)(hi - lo) * (part + 1) / parts);
                for (int j = a; j < b; ++j) {
                    const double* q = qg + 24 * (size_t)j + 3 * (kk - (sv[j] - prof.p));
                    acc = acc + mk(q[0], q[1], q[2]);
                }
                if (!prof.closed) break;
            }
            if (parts == 1) {
                double* o = gQ + 3 * (d.prof_ctrl_off + l);
                o[0] = acc.x; o[1] = acc.y; o[2] = acc.z;
            } else {
                lpart[t][0] = acc.x; lpart[t][1] = acc.y; lpart[t][2] = acc.z;
            }
        }
        __syncthreads();
        if (parts > 1)
            for (int l = threadIdx.x; l < d.n_prof; l += kBlock) {
                V3<double> acc = mk(0.0, 0.0, 0.0);
                for (int part = 0; part < parts; ++part)
                    acc = acc + mk(lpart[l * parts + part][0], lpart[l * parts + part][1], lpart[l * parts + part][2]);
                double* o = gQ + 3 * (d.prof_ctrl_off + l);
                o[0] = acc.x; o[1] = acc.y; o[2] = acc.z;
            }
    }
}

// ------------------------------------------------ knot and weight gradients

// Per-sample records of the parameter gradients (kParamRec doubles): the
// 2p local knot contributions, then the p+1 local weight contributions, and
// dL/du (the sample's parameter) in the last slot.
constexpr int kParamRec = 24;

// Contributions of one sample on span s at parameter u, given dL/dC, dL/dC'
// and dL/dC'' there: kc[m] = dL/dU_{s-P+1+m} at fixed u (m < 2P), wc[l] =
// dL/dw_{s-P+l} (rational curves), and the return value dL/du.  Dual-number
// passes of the basis and curve derivatives, one per local knot or weight.
template <int P>
__device__ __noinline__ double param_contrib(const DCurve& c, double u, int s, V3<double> xb, V3<double> cb,
                                             V3<double> c2b, bool want_k, bool want_w, double* kc, double* wc)
{
    double Pl[P + 1][3];
    Dual Ud[2 * P], wd[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        const V3<double> q = ctrl_pt(c, s - P + j);
        Pl[j][0] = q.x; Pl[j][1] = q.y; Pl[j][2] = q.z;
        wd[j] = dual(c.w ? weight_at(c, s - P + j) : 1.0);
    }
#pragma unroll
    for (int m = 0; m < 2 * P; ++m) Ud[m] = dual(knot(c, s - P + 1 + m));
    const Dual* wp = c.w ? wd : nullptr;
    const Dual ud = dual(u);
    // dL/du: C', C'', C''' at fixed knots and weights
    double eu;
    {
        Dual D[4][P + 1], C[4][3];
        basis_ders<P, 3, Dual>(Ud, ud, D);
        curve_ders<P, 3, Dual>(D, Pl, wp, C);
        eu = xb.x * C[1][0].v + xb.y * C[1][1].v + xb.z * C[1][2].v + cb.x * C[2][0].v + cb.y * C[2][1].v +
             cb.z * C[2][2].v + c2b.x * C[3][0].v + c2b.y * C[3][1].v + c2b.z * C[3][2].v;
    }
    auto contract = [&](const Dual (&C)[3][3]) {
        return xb.x * C[0][0].d + xb.y * C[0][1].d + xb.z * C[0][2].d + cb.x * C[1][0].d + cb.y * C[1][1].d +
               cb.z * C[1][2].d + c2b.x * C[2][0].d + c2b.y * C[2][1].d + c2b.z * C[2][2].d;
    };
    if (want_k) {
        for (int m = 0; m < 2 * P; ++m) {
            Ud[m].d = 1.0;
            Dual D[3][P + 1], C[3][3];
            basis_ders<P, 2, Dual>(Ud, ud, D);
            curve_ders<P, 2, Dual>(D, Pl, wp, C);
            kc[m] = contract(C);
            Ud[m].d = 0.0;
        }
    }
    if (want_w && c.w) {
        Dual D[3][P + 1];
        basis_ders<P, 2, Dual>(Ud, ud, D);
        for (int l = 0; l <= P; ++l) {
            wd[l].d = 1.0;
            Dual C[3][3];
            curve_ders<P, 2, Dual>(D, Pl, wd, C);
            wc[l] = contract(C);
            wd[l].d = 0.0;
        }
    }
    return eu;
}

__device__ __forceinline__ double param_contrib_any(const DCurve& c, double u, int s, V3<double> xb, V3<double> cb,
                                                    V3<double> c2b, bool want_k, bool want_w, double* kc,
                                                    double* wc)
{
    switch (c.p) {
    case 1: return param_contrib<1>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    case 2: return param_contrib<2>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    case 3: return param_contrib<3>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    case 4: return param_contrib<4>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    case 5: return param_contrib<5>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    case 6: return param_contrib<6>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    default: return param_contrib<7>(c, u, s, xb, cb, c2b, want_k, want_w, kc, wc);
    }
}

// Sum over the block of (a, b) pairs, thread order fixed.
__device__ __forceinline__ void block_pair_total(double a, double b, double (*lds)[3], double& ta, double& tb)
{
    V3<double> tot;
    block_suffix_sum(mk(a, b, 0.0), lds, tot);
    ta = tot.x;
    tb = tot.y;
}

// One curve's knot and weight gradients from its per-sample records
// (kbw_param_rec): the domain-end terms of the sample parameters
// (u = U_p + (U_n - U_p) i/(ns-1) on an open curve), then one thread per
// knot / weight gathers the samples whose span reaches it.
__device__ void curve_param_grads(const DCurve& c, int ns, const int* spans, const double* rec, bool want_k,
                                  bool want_w, double* gk, double* gw, double (*lds)[3], double* lpart)
{
    const int p = c.p;
    double e0 = 0.0, e1 = 0.0;   // dL/dU_p and dL/dU_n through the sample parameters
    if (want_k) {
        for (int b0 = 0; b0 < ns; b0 += kBlock) {
            const int i = b0 + threadIdx.x;
            double a = 0.0, b = 0.0;
            if (i < ns) {
                const double eu = rec[kParamRec * (size_t)i + kParamRec - 1];
                const double f = (double)i / (double)(ns - 1);
                a = eu * (1.0 - f);
                b = eu * f;
            }
            double ta, tb;
            block_pair_total(a, b, lds, ta, tb);
            e0 += ta;
            e1 += tb;
        }
        // knots 0 .. n+p: samples with span in [m-p, m+p-1] reach knot m;
        // `parts` threads per knot each sum a contiguous piece of that range,
        // the pieces added in part order
        const int nk = c.n + p + 1;
        const int parts = nk <= kBlock ? min(kMaxParts, kBlock / nk) : 1;
        for (int t = threadIdx.x; t < nk * parts; t += kBlock) {
            const int m = t / parts, part = t % parts;
            const int lo = lower_bound_int(spans, ns, m - p), hi = lower_bound_int(spans, ns, m + p);
            const int a = lo + (int)((long long)(hi - lo) * part / parts);
            const int b = lo + (int)((long long)(hi - lo) * (part + 1) / parts);
            double acc = 0.0;
            for (int i = a; i < b; ++i) acc += rec[kParamRec * (size_t)i + (m - (spans[i] - p + 1))];
            if (parts == 1) {
                if (m == p) acc += e0;
                if (m == c.n) acc += e1;
                gk[m] = acc;
            } else {
                lpart[t] = acc;
            }
        }
        __syncthreads();
        if (parts > 1)
            for (int m = threadIdx.x; m < nk; m += kBlock) {
                double acc = 0.0;
                for (int part = 0; part < parts; ++part) acc += lpart[m * parts + part];
                if (m == p) acc += e0;
                if (m == c.n) acc += e1;
                gk[m] = acc;
            }
        __syncthreads();
    }
    if (want_w && c.w) {
        // weight l: basis indices l (and l + n on a closed curve), reached by
        // the samples with span in [k, k+p]
        const int parts = c.n <= kBlock ? min(kMaxParts, kBlock / c.n) : 1;
        for (int t = threadIdx.x; t < c.n * parts; t += kBlock) {
            const int l = t / parts, part = t % parts;
            double acc = 0.0;
            for (int kk = l; kk < c.nb; kk += c.n) {
                const int lo = lower_bound_int(spans, ns, kk), hi = lower_bound_int(spans, ns, kk + p + 1);
                const int a = lo + (int)((long long)(hi - lo) * part / parts);
                const int b = lo + (int)((long long)(hi - lo) * (part + 1) / parts);
                for (int i = a; i < b; ++i) acc += rec[kParamRec * (size_t)i + 2 * p + (kk - (spans[i] - p))];
                if (!c.closed) break;
            }
            if (parts == 1) gw[l] = acc;
            else lpart[t] = acc;
        }
        __syncthreads();
        if (parts > 1)
            for (int l = threadIdx.x; l < c.n; l += kBlock) {
                double acc = 0.0;
                for (int part = 0; part < parts; ++part) acc += lpart[l * parts + part];
                gw[l] = acc;
            }
    }
    __syncthreads();
}

// Per-sample records of the knot and weight gradients: one block per
// (sweep, chunk of kBlock samples) of the path (PROFILE false: adjoints from
// xstash, dL/dC, dL/dC', dL/dC'' per sample, written by kbw_samples) or of
// the profile (PROFILE true: dL/dS and dL/dS' from colacc).
template <bool PROFILE>
__global__ __launch_bounds__(kBlock) void kbw_param_rec(const BatchDesc* __restrict__ descs,
                                                        const int2* __restrict__ chunks,
                                                        const double* __restrict__ path_ctrl,
                                                        const double* __restrict__ prof_ctrl,
                                                        const double* __restrict__ path_w,
                                                        const double* __restrict__ prof_w,
                                                        const double* __restrict__ knots, const double* xstash,
                                                        const double* colacc, const int* spans_u,
                                                        const int* spans_v, double* recu, double* recv, int nrm,
                                                        int want_k, int want_w)
{
    const int2 ch = chunks[blockIdx.x];
    const BatchDesc d = descs[ch.x];
    const int i = ch.y * kBlock + threadIdx.x;
    const int ns = PROFILE ? d.n_v : d.n_u;
    const bool wk = want_k && (PROFILE ? d.prof_kuser_off : d.path_kuser_off) >= 0;
    if (i >= ns || !(wk || want_w)) return;
    const DCurve c = PROFILE
        ? DCurve{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr, d.n_prof,
                 d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof,
                 prof_w ? prof_w + d.prof_ctrl_off : nullptr}
        : DCurve{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr, d.n_path,
                 d.p_path, 0, d.n_path, path_w ? path_w + d.path_ctrl_off : nullptr};
    V3<double> xb, cb, c2b = mk(0.0, 0.0, 0.0);
    if (PROFILE) {
        const int cp = nrm ? kColPartNrm : kColPart;
        const double* q = colacc + (size_t)cp * (d.ptab_off + i);
        xb = mk(q[0], q[1], q[2]);
        cb = nrm ? mk(q[3], q[4], q[5]) : mk(0.0, 0.0, 0.0);
    } else {
        const double* q = xstash + 9 * (d.row_off + (size_t)i);
        xb = mk(q[0], q[1], q[2]);
        cb = mk(q[3], q[4], q[5]);
        c2b = mk(q[6], q[7], q[8]);
    }
    const size_t o = PROFILE ? d.ptab_off : d.row_off;
    double* r = (PROFILE ? recv : recu) + kParamRec * (o + i);
    const int s = (PROFILE ? spans_v : spans_u)[o + i];
    r[kParamRec - 1] = param_contrib_any(c, sample_param(c, i, ns), s, xb, cb, c2b, wk, want_w, r, r + 2 * c.p);
}

// One block per sweep, after kbw_param_rec: the domain-end terms and the
// gathers per knot and weight.
__global__ __launch_bounds__(kBlock) void kbw_params(const BatchDesc* __restrict__ descs,
                                                     const double* __restrict__ path_ctrl,
                                                     const double* __restrict__ prof_ctrl,
                                                     const double* __restrict__ path_w,
                                                     const double* __restrict__ prof_w,
                                                     const double* __restrict__ knots, const int* spans_u,
                                                     const int* spans_v, const double* recu, const double* recv,
                                                     double* gPk, double* gQk, double* gPw, double* gQw)
{
    __shared__ double lds3[kWaves][3];
    __shared__ double lpart[kBlock];
    const BatchDesc d = descs[blockIdx.x];
    const DCurve path{path_ctrl + 3 * d.path_ctrl_off, d.path_knot_off >= 0 ? knots + d.path_knot_off : nullptr,
                      d.n_path, d.p_path, 0, d.n_path, path_w ? path_w + d.path_ctrl_off : nullptr};
    const DCurve prof{prof_ctrl + 3 * d.prof_ctrl_off, d.prof_knot_off >= 0 ? knots + d.prof_knot_off : nullptr,
                      d.n_prof, d.p_prof, d.closed_prof, d.closed_prof ? d.n_prof + d.p_prof : d.n_prof,
                      prof_w ? prof_w + d.prof_ctrl_off : nullptr};
    const bool pk = gPk && d.path_kuser_off >= 0, qk = gQk && d.prof_kuser_off >= 0;
    const bool pw = gPw != nullptr, qw = gQw != nullptr;
    if (pk || pw)
        curve_param_grads(path, d.n_u, spans_u + d.row_off, recu + kParamRec * d.row_off, pk, pw,
                          pk ? gPk + d.path_kuser_off : nullptr, pw ? gPw + d.path_ctrl_off : nullptr, lds3, lpart);
    if (qk || qw)
        curve_param_grads(prof, d.n_v, spans_v + d.ptab_off, recv + kParamRec * d.ptab_off, qk, qw,
                          qk ? gQk + d.prof_kuser_off : nullptr, qw ? gQw + d.prof_ctrl_off : nullptr, lds3, lpart);
}

BackwardKernels backward_kernels(bool t64, bool nrm)
{
    BackwardKernels k;
    if (nrm) k.reduce = t64 ? (const void*)&kbw_reduce<double, true> : (const void*)&kbw_reduce<float, true>;
    else k.reduce = t64 ? (const void*)&kbw_reduce<double, false> : (const void*)&kbw_reduce<float, false>;
    k.rows = (const void*)&kbw_rows;
    k.samples = (const void*)&kbw_samples;
    k.final_ = (const void*)&kbw_final;
    k.params = (const void*)&kbw_params;
    k.param_rec_path = (const void*)&kbw_param_rec<false>;
    k.param_rec_prof = (const void*)&kbw_param_rec<true>;
    return k;
}

}  // namespace sweep
