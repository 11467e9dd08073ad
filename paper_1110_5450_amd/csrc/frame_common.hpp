// frame_common.hpp -- device steps of the frame computation shared by the
// single-sweep kernels (frame_kernels.hip) and the batched kernel
// (batched_kernels.hip): tangents, the initial normal, the chunk carry scan,
// row records and profile records.
#pragma once

#include "device_math.hpp"
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace sweep {

// d/|d| (one division for the three components).
__device__ __forceinline__ V3<double> unit_of(V3<double> d)
{
    const double inv = recip(sqrt(dot(d, d)));
    return inv * d;
}

// Initial normal r_0 from the resolved t_0: the given normal projected onto
// t_0^perp when that projection exceeds 1e-8, else the axis rule.
__device__ __forceinline__ V3<double> initial_normal(V3<double> t0, const InitialNormal& n0)
{
    if (n0.enabled) {
        const V3<double> n = mk(n0.v[0], n0.v[1], n0.v[2]);
        const V3<double> q = n - dot(n, t0) * t0;
        const double L = sqrt(dot(q, q));
        if (L > 1e-8) return divs(q, L);
    }
    return axis_normal(t0);
}

// r_in[c] = (A_{c-1} ... A_0) r_0 for c < n_chunks, by one block (all threads).
template <class F>
__device__ void carry_scan(const F* agg, int n_chunks, V3<double> r0d, F* __restrict__ r_in, M3<F>* lds_m)
{
    const V3<F> r0 = cvt<F>(r0d);
    constexpr int kPer = 4;
    M3<F> running = ident<F>();
    for (int base = 0; base < n_chunks; base += kBlock * kPer) {
        M3<F> A[kPer];
        M3<F> prod = ident<F>();
        const int c0 = base + threadIdx.x * kPer;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int c = c0 + k;
            if (c < n_chunks) {
#pragma unroll
                for (int e = 0; e < 9; ++e) A[k].m[e] = __builtin_nontemporal_load(agg + 9 * (size_t)c + e);
            } else {
                A[k] = ident<F>();
            }
            prod = mul(A[k], prod);
        }
        M3<F> total;
        M3<F> ex = mul(block_exclusive_product<F>(prod, lds_m, total), running);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
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

// Row record of one sample: x, r (re-orthonormalised against t if asked),
// s = t x r, t, |C'|, a = r.C''/|C'|, b = s.C''/|C'| (0 where C' = 0), in
// precision T.  r is the carried normal in the frame precision F.
template <class F, class T>
__device__ __forceinline__ void write_row(V3<double> x, V3<double> td, V3<F> r, V3<double> C1, V3<double> C2,
                                          int reorth, T* __restrict__ q)
{
    const V3<F> t = cvt<F>(td);
    if (reorth) {
        const V3<F> w = r - dot(r, t) * t;
        r = recip((F)sqrt(dot(w, w))) * w;
    }
    const V3<F> sv = cross(t, r);
    const double L = sqrt(dot(C1, C1));
    F a = F(0), b = F(0);
    if (L > 0.0) {
        const V3<F> c2 = cvt<F>(C2);
        const F inv = recip((F)L);
        a = dot(r, c2) * inv;
        b = dot(sv, c2) * inv;
    }
    q[0] = (T)x.x; q[1] = (T)x.y; q[2] = (T)x.z;
    q[3] = (T)r.x; q[4] = (T)r.y; q[5] = (T)r.z;
    q[6] = (T)sv.x; q[7] = (T)sv.y; q[8] = (T)sv.z;
    q[9] = (T)t.x; q[10] = (T)t.y; q[11] = (T)t.z;
    q[12] = (T)L; q[13] = (T)a; q[14] = (T)b; q[15] = T(0);
}

// ------------------------------------------------ frame modes and laws

// Extended row record (kRowExt values), used with the Frenet frame mode or a
// sweep law: x (3), r (3), s (3), t (3), |C'|, a, b, omega, A (2x2 row-major),
// A' (2x2), sigma, sigma', 0 x 6.  omega is the rate (per unit u) at which
// the frame turns about t relative to a rotation-minimizing one (0 for the
// rotation-minimizing frame, |C'| tau for Frenet); A = sigma Rot(theta) maps
// the profile's (x, y) into the (r, s) plane, A' = dA/du; sigma scales the
// profile's z.  (kRowExt is declared with the launchers.)

// Relative size below which C'' has no component normal to t (no Frenet
// normal: the axis rule is used and omega = 0).
constexpr double kFrenetEps = 1e-8;

// Law value at a u-sample: scale, twist angle and their u-derivatives.
struct LawSample {
    double sg, th, dsg, dth;
};

template <class F, class T>
__device__ __forceinline__ void write_row_ext(V3<double> x, V3<double> td, V3<F> rc, V3<double> C1, V3<double> C2,
                                              V3<double> C3, int frenet, LawSample lw, int reorth, T* __restrict__ q)
{
    const V3<F> t = cvt<F>(td);
    V3<F> r;
    double omega = 0.0;
    if (frenet) {
        // principal normal from C'' (pointwise, FP64), torsion rate from C'''
        const double ct = dot(C2, td);
        const V3<double> qv = C2 - ct * td;
        const double nq = sqrt(dot(qv, qv));
        V3<double> rd;
        if (nq > kFrenetEps * sqrt(dot(C2, C2))) {
            rd = divs(qv, nq);
            const V3<double> k = cross(C1, C2);
            const double kk = dot(k, k);
            if (kk > 0.0) omega = sqrt(dot(C1, C1)) * (dot(k, C3) / kk);
        } else {
            rd = axis_normal<double>(td);
        }
        r = cvt<F>(rd);
    } else {
        r = rc;
        if (reorth) {
            const V3<F> w = r - dot(r, t) * t;
            r = recip((F)sqrt(dot(w, w))) * w;
        }
    }
    const V3<F> sv = cross(t, r);
    const double L = sqrt(dot(C1, C1));
    F a = F(0), b = F(0);
    if (L > 0.0) {
        const V3<F> c2 = cvt<F>(C2);
        const F inv = recip((F)L);
        a = dot(r, c2) * inv;
        b = dot(sv, c2) * inv;
    }
    const double c = cos(lw.th), sn = sin(lw.th);
    q[0] = (T)x.x; q[1] = (T)x.y; q[2] = (T)x.z;
    q[3] = (T)r.x; q[4] = (T)r.y; q[5] = (T)r.z;
    q[6] = (T)sv.x; q[7] = (T)sv.y; q[8] = (T)sv.z;
    q[9] = (T)t.x; q[10] = (T)t.y; q[11] = (T)t.z;
    q[12] = (T)L; q[13] = (T)a; q[14] = (T)b; q[15] = (T)omega;
    q[16] = (T)(lw.sg * c); q[17] = (T)(-lw.sg * sn); q[18] = (T)(lw.sg * sn); q[19] = (T)(lw.sg * c);
    const double gc = lw.dsg * c - lw.sg * lw.dth * sn, gs = lw.dsg * sn + lw.sg * lw.dth * c;
    q[20] = (T)gc; q[21] = (T)(-gs); q[22] = (T)gs; q[23] = (T)gc;
    q[24] = (T)lw.sg; q[25] = (T)lw.dsg;
#pragma unroll
    for (int e = 26; e < kRowExt; ++e) q[e] = T(0);
}

// Law at u-sample i of n_u: the law curve holds (sigma, theta, -) and is
// sampled like the path; dl/du = du_scale.  No law: sigma = 1, theta = 0.
__device__ __forceinline__ LawSample law_at(const DCurve* law, int i, int n_u, double du_scale)
{
    LawSample lw{1.0, 0.0, 0.0, 0.0};
    if (law) {
        V3<double> o[2];
        sample_derivs_any<1>(*law, i, n_u, o);
        lw.sg = o[0].x; lw.th = o[0].y;
        lw.dsg = o[1].x * du_scale; lw.dth = o[1].y * du_scale;
    }
    return lw;
}

// C and C' of a curve of any degree p <= kMaxDeg at sample j of ns, with loops
// over the run-time degree instead of one unrolled copy per degree: the same
// operations in the same order as curve_derivs<P, 1>, on local arrays.  Used
// for the profile tables, which are small and evaluated once per call, so
// that the kernels holding them do not reserve the registers of an unrolled
// degree-7 evaluation.
__device__ __forceinline__ void curve_d1_any(const DCurve& c, int j, int ns, V3<double>* out)
{
    const int p = c.p;
    double u;
    int s;
    if (c.su) {
        u = c.su[j];
        s = c.ss[j];
    } else {
        u = sample_param(c, j, ns);
        s = sample_span(c, j, ns, u);
    }
    double Uk[2 * kMaxDeg];
#pragma unroll 1
    for (int m = 0; m < 2 * p; ++m) Uk[m] = knot(c, s - p + 1 + m);
    double B[kMaxDeg + 1], D1[kMaxDeg + 1], nb_[kMaxDeg + 1];
    B[0] = 1.0;
    D1[0] = 1.0;
#pragma unroll 1
    for (int q = 1; q <= p; ++q) {
        double carry = 0.0;
#pragma unroll 1
        for (int k = 0; k < q; ++k) {
            const double lo = Uk[p - q + k], hi = Uk[p + k];
            const double tmp = B[k] / (hi - lo);
            nb_[k] = carry + (hi - u) * tmp;
            carry = (u - lo) * tmp;
        }
        nb_[q] = carry;
#pragma unroll 1
        for (int k = 0; k <= q; ++k) B[k] = nb_[k];
        if (q == p - 1) {
#pragma unroll 1
            for (int k = 0; k <= q; ++k) D1[k] = B[k];
        }
    }
    V3<double> C0 = mk(0.0, 0.0, 0.0), C1 = C0;
    if (!c.w) {
#pragma unroll 1
        for (int k = 0; k <= p; ++k) C0 = C0 + B[k] * ctrl_pt(c, s - p + k);
#pragma unroll 1
        for (int k = 0; k < p; ++k)
            C1 = C1 + D1[k] * (((double)p / (Uk[p + k] - Uk[k])) * (ctrl_pt(c, s - p + k + 1) - ctrl_pt(c, s - p + k)));
    } else {
        // homogeneous curve (w P, w) and the quotient rule
        double W0 = 0.0, W1 = 0.0;
#pragma unroll 1
        for (int k = 0; k <= p; ++k) {
            const double wk = weight_at(c, s - p + k);
            C0 = C0 + B[k] * (wk * ctrl_pt(c, s - p + k));
            W0 = W0 + B[k] * wk;
        }
        V3<double> A1 = mk(0.0, 0.0, 0.0);
#pragma unroll 1
        for (int k = 0; k < p; ++k) {
            const double f = (double)p / (Uk[p + k] - Uk[k]);
            const double w0 = weight_at(c, s - p + k), w1 = weight_at(c, s - p + k + 1);
            A1 = A1 + D1[k] * (f * (w1 * ctrl_pt(c, s - p + k + 1) - w0 * ctrl_pt(c, s - p + k)));
            W1 = W1 + D1[k] * (f * (w1 - w0));
        }
        C0 = divs(C0, W0);
        C1 = divs(A1 - W1 * C0, W0);
    }
    out[0] = C0;
    out[1] = C1;
}

// Profile record of sample j: S (3), S' (3), 0, 0.
template <class T>
__device__ __forceinline__ void write_profile(const DCurve& prof, int j, int n_v, T* __restrict__ tab)
{
    V3<double> o[2];
    curve_d1_any(prof, j, n_v, o);
    T* q = tab + 8 * (size_t)j;
    q[0] = (T)o[0].x; q[1] = (T)o[0].y; q[2] = (T)o[0].z;
    q[3] = (T)o[1].x; q[4] = (T)o[1].y; q[5] = (T)o[1].z;
    q[6] = T(0); q[7] = T(0);
}

// Unit direction of the first nonzero control-polygon leg, else e_z.
__device__ __forceinline__ V3<double> first_leg(const DCurve& path)
{
    for (int k = 0; k + 1 < path.n; ++k) {
        const V3<double> d = ctrl_pt(path, k + 1) - ctrl_pt(path, k);
        const double L2 = dot(d, d);
        if (L2 > 0.0) return divs(d, sqrt(L2));
    }
    return mk(0.0, 0.0, 1.0);
}

}  // namespace sweep

// back to the default (contraction across statements) for code that follows
#pragma clang fp contract(fast)
