// device_math.hpp -- small vector/matrix types and the B-spline evaluation
// used by the sweep kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// FP contraction is off for everything in this header and frame_common.hpp
// (curve evaluation, step rotations, block products): each product and sum
// is rounded where written, so a function inlined into different kernels
// gives bitwise identical results (single-sweep and batched paths agree).
#pragma clang fp contract(off)

namespace sweep {

constexpr int kBlock = 256;   // threads per block in every kernel
constexpr int kWaves = kBlock / 64;
constexpr int kMaxDeg = 7;

template <class F> struct V3 { F x, y, z; };

template <class F> __device__ __forceinline__ V3<F> mk(F x, F y, F z) { return V3<F>{x, y, z}; }
template <class F> __device__ __forceinline__ V3<F> operator+(V3<F> a, V3<F> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class F> __device__ __forceinline__ V3<F> operator-(V3<F> a, V3<F> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class F> __device__ __forceinline__ V3<F> operator*(F s, V3<F> a) { return {s * a.x, s * a.y, s * a.z}; }
// dot and cross products as explicit fused multiply-adds (the rounding does
// not depend on where they are inlined)
template <class F> __device__ __forceinline__ F dot(V3<F> a, V3<F> b) { return fma(a.z, b.z, fma(a.y, b.y, a.x * b.x)); }
template <class F> __device__ __forceinline__ V3<F> cross(V3<F> a, V3<F> b)
{
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}
// s a + b, componentwise fused
template <class F> __device__ __forceinline__ V3<F> fmadd(F s, V3<F> a, V3<F> b)
{
    return {fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z)};
}
template <class F> __device__ __forceinline__ V3<F> divs(V3<F> a, F s) { return {a.x / s, a.y / s, a.z / s}; }
template <class G, class F> __device__ __forceinline__ V3<G> cvt(V3<F> a) { return {(G)a.x, (G)a.y, (G)a.z}; }

// 3x3 matrix, row-major.
template <class F> struct M3 { F m[9]; };

template <class F> __device__ __forceinline__ M3<F> ident()
{
    M3<F> r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.m[k] = (k % 4 == 0) ? F(1) : F(0);
    return r;
}
// a * b, each entry as two fused multiply-adds (explicit, so the rounding
// does not depend on where the function is inlined)
template <class F> __device__ __forceinline__ M3<F> mul(const M3<F>& a, const M3<F>& b)
{
    M3<F> r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r.m[3 * i + j] = fma(a.m[3 * i + 2], b.m[6 + j], fma(a.m[3 * i + 1], b.m[3 + j], a.m[3 * i] * b.m[j]));
    return r;
}
template <class F> __device__ __forceinline__ V3<F> apply(const M3<F>& a, V3<F> v)
{
    return {fma(a.m[2], v.z, fma(a.m[1], v.y, a.m[0] * v.x)),
            fma(a.m[5], v.z, fma(a.m[4], v.y, a.m[3] * v.x)),
            fma(a.m[8], v.z, fma(a.m[7], v.y, a.m[6] * v.x))};
}

// 1/x from the hardware reciprocal refined by Newton steps (two in FP64, one
// in FP32): within an ulp or two of the correctly rounded quotient, with a
// shorter dependency chain than the IEEE division, and the same instructions
// wherever it is inlined.  No branch: where the refinement is not finite
// (x = 0, inf, NaN, or a quotient beyond the range) the hardware value is
// the result (inf, 0, NaN or inf).  Denormal x gives inf in FP64 (as the
// hardware reciprocal does).
__device__ __forceinline__ double recip(double x)
{
    const double r0 = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r0, 1.0);
    double r = fma(r0, e, r0);
    e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    return __builtin_isfinite(r) ? r : r0;
}
__device__ __forceinline__ float recip(float x)
{
    const float r0 = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r0, 1.0f);
    const float r = fmaf(r0, e, r0);
    return __builtin_isfinite(r) ? r : r0;
}

// ------------------------------------------------------------------ curves

struct DCurve {
    const double* __restrict__ ctrl;   // n x 3
    const double* __restrict__ knots;  // nb + p + 1 given knots, or nullptr for the default vector
    int n;       // distinct control points
    int p;       // degree
    int closed;  // periodic uniform
    int nb;      // basis functions: n (open) or n + p (closed)
    const double* __restrict__ w;      // n weights (rational curve), or nullptr
    const double* __restrict__ su;     // sample parameters (arc-length sampling), or nullptr
    const int* __restrict__ ss;        // their spans
};

__device__ __forceinline__ V3<double> ctrl_pt(const DCurve& c, int k)
{
    const int kk = (c.closed && k >= c.n) ? k - c.n : k;
    const double* q = c.ctrl + 3 * (size_t)kk;
    return {q[0], q[1], q[2]};
}

__device__ __forceinline__ double weight_at(const DCurve& c, int k)
{
    return c.w[(c.closed && k >= c.n) ? k - c.n : k];
}

// Knot k: the given vector, else periodic U_k = k, else clamped uniform
// 0 (k <= p), 1 (k >= n), (k-p)/(n-p) as one correctly rounded division.
__device__ __forceinline__ double knot(const DCurve& c, int k)
{
    if (c.knots) return c.knots[k];
    if (c.closed) return (double)k;
    if (k <= c.p) return 0.0;
    if (k >= c.n) return 1.0;
    return (double)(k - c.p) / (double)(c.n - c.p);
}

// Sample parameter i of ns.  Open: u = a + (b - a) * (i / (ns - 1)), with the
// last sample exactly b; closed: p + (n*i)/ns.  Each operation is rounded as
// written (no contraction), so samples that fall on a knot land on it exactly.
__device__ __forceinline__ double sample_param(const DCurve& c, int i, int ns)
{
#pragma clang fp contract(off)
    if (c.closed) return (double)c.p + (double)((long long)c.n * (long long)i) / (double)ns;
    const double a = knot(c, c.p), b = knot(c, c.n);
    if (i == ns - 1) return b;
    const double f = (double)i / (double)(ns - 1);
    const double w = b - a;
    const double g = w * f;
    return a + g;
}

// Span of sample i: the largest k in [p, nb-1] with U_k <= u (nb-1 at the
// right end).  For the default knots the comparison U_k <= u_i is a
// comparison of two correctly rounded quotients of small integers, which
// agrees with the comparison of the exact rationals, so the span follows
// from integer arithmetic: p + floor(i (n-p) / (ns-1)) (open) or
// p + floor(n i / ns) (closed).  Given knots: binary search.
__device__ __forceinline__ int sample_span(const DCurve& c, int i, int ns, double u)
{
    if (!c.knots) {
        if (c.closed) return c.p + (int)(((long long)c.n * (long long)i) / ns);
        const int s = c.p + (int)(((long long)i * (long long)(c.n - c.p)) / (ns - 1));
        return s < c.n - 1 ? s : c.n - 1;
    }
    const double* __restrict__ U = c.knots;
    if (u >= U[c.nb]) return c.nb - 1;
    int lo = c.p, hi = c.nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (U[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Rational curve (NURBS Book ch. 4): the homogeneous curve (w P, w) has the
// same basis and derivative nets, giving A, A', A'' and W, W', W''; then
// C = A / W, C' = (A' - W' C) / W, C'' = (A'' - 2 W' C' - W'' C) / W, and
// the third derivative C3 = (A3 - 3 W' C'' - 3 W'' C' - W3 C) / W.
// Uk, B, D1, D2 as in curve_derivs; Pt the P+1 control points of span s.
template <int P, int ND>
__device__ __forceinline__ void rational_derivs(const DCurve& c, int s, const double* Uk, const double* B,
                                                const double* D1, const double* D2, const double* D3,
                                                const V3<double>* Pt, V3<double>* out)
{
    V3<double> Hw[P + 1];
    double wt[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        wt[j] = weight_at(c, s - P + j);
        Hw[j] = wt[j] * Pt[j];
    }
    V3<double> A0 = mk(0.0, 0.0, 0.0);
    double W0 = 0.0;
#pragma unroll
    for (int j = 0; j <= P; ++j) { A0 = A0 + B[j] * Hw[j]; W0 = W0 + B[j] * wt[j]; }
    const V3<double> C0 = divs(A0, W0);
    out[0] = C0;
    if (ND >= 1) {
        V3<double> Q1[P > 0 ? P : 1];
        double q1[P > 0 ? P : 1];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double f = (double)P / (Uk[P + j] - Uk[j]);
            Q1[j] = f * (Hw[j + 1] - Hw[j]);
            q1[j] = f * (wt[j + 1] - wt[j]);
        }
        V3<double> A1 = mk(0.0, 0.0, 0.0);
        double W1 = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) { A1 = A1 + D1[j] * Q1[j]; W1 = W1 + D1[j] * q1[j]; }
        const V3<double> C1 = divs(A1 - W1 * C0, W0);
        out[1] = C1;
        if (ND >= 2) {
            V3<double> A2 = mk(0.0, 0.0, 0.0);
            double W2 = 0.0;
            V3<double> Q2[P > 1 ? P - 1 : 1];
            double q2[P > 1 ? P - 1 : 1];
            if (P >= 2) {
#pragma unroll
                for (int j = 0; j + 1 < P; ++j) {
                    const double f = (double)(P - 1) / (Uk[P + j] - Uk[j + 1]);
                    Q2[j] = f * (Q1[j + 1] - Q1[j]);
                    q2[j] = f * (q1[j + 1] - q1[j]);
                    A2 = A2 + D2[j] * Q2[j];
                    W2 = W2 + D2[j] * q2[j];
                }
            }
            const V3<double> C2 = divs(A2 - (2.0 * W1) * C1 - W2 * C0, W0);
            out[2] = C2;
            if (ND >= 3) {
                V3<double> A3 = mk(0.0, 0.0, 0.0);
                double W3 = 0.0;
                if (P >= 3) {
#pragma unroll
                    for (int j = 0; j + 2 < P; ++j) {
                        const double f = (double)(P - 2) / (Uk[P + j] - Uk[j + 2]);
                        A3 = A3 + D3[j] * (f * (Q2[j + 1] - Q2[j]));
                        W3 = W3 + D3[j] * (f * (q2[j + 1] - q2[j]));
                    }
                }
                out[3] = divs(A3 - (3.0 * W1) * C2 - (3.0 * W2) * C1 - W3 * C0, W0);
            }
        }
    }
}

// C and derivatives up to order ND at u (in span s) for a degree-P B-spline
// (rational when c.w is set).
// Basis values of degrees P, P-1, P-2 come from one triangular sweep of the
// Cox-de Boor recursion (one division per knot interval and degree);
// derivatives use the derivative control nets
//   Q_k = P (P_{k+1} - P_k) / (U_{k+P+1} - U_{k+1}),
//   R_k = (P-1)(Q_{k+1} - Q_k) / (U_{k+P+1} - U_{k+2}),
// whose denominators are positive on a non-empty span.
template <int P, int ND>
__device__ __forceinline__ void curve_derivs(const DCurve& c, double u, int s, V3<double>* out)
{
    double Uk[2 * P + 1];   // U_{s-P+1+m}, m = 0..2P-1 (index 2P unused)
#pragma unroll
    for (int m = 0; m < 2 * P; ++m) Uk[m] = knot(c, s - P + 1 + m);
#define UK(k) Uk[(k) - (s - P + 1)]
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
        // B holds N_{s-q+1+j, q-1}, j = 0..q-1; build N_{s-q+j, q}, j = 0..q.
        double nb_[P + 1];
        double carry = 0.0;
#pragma unroll
        for (int j = 0; j < q; ++j) {
            const double lo = Uk[P - q + j], hi = Uk[P + j];   // U_{s-q+j+1}, U_{s+j+1}
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
        if (ND >= 3 && q == P - 3) {
#pragma unroll
            for (int j = 0; j <= q; ++j) D3[j] = B[j];
        }
    }
    V3<double> Pt[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) Pt[j] = ctrl_pt(c, s - P + j);
    if (c.w) {
        rational_derivs<P, ND>(c, s, Uk, B, D1, D2, D3, Pt, out);
        return;
    }
    V3<double> C0 = mk(0.0, 0.0, 0.0);
#pragma unroll
    for (int j = 0; j <= P; ++j) C0 = C0 + B[j] * Pt[j];
    out[0] = C0;
    if (ND >= 1) {
        V3<double> Q1[P > 0 ? P : 1];
#pragma unroll
        for (int j = 0; j < P; ++j) Q1[j] = ((double)P / (Uk[P + j] - Uk[j])) * (Pt[j + 1] - Pt[j]);
        V3<double> C1 = mk(0.0, 0.0, 0.0);
#pragma unroll
        for (int j = 0; j < P; ++j) C1 = C1 + D1[j] * Q1[j];
        out[1] = C1;
        if (ND >= 2) {
            V3<double> C2 = mk(0.0, 0.0, 0.0);
            V3<double> R2[P > 1 ? P - 1 : 1];
            if (P >= 2) {
#pragma unroll
                for (int j = 0; j + 1 < P; ++j) {
                    const V3<double> R = ((double)(P - 1) / (Uk[P + j] - Uk[j + 1])) * (Q1[j + 1] - Q1[j]);
                    C2 = C2 + D2[j] * R;
                    R2[j] = R;
                }
            }
            out[2] = C2;
            if (ND >= 3) {
                // third derivative net (P-2)(R_{k+1} - R_k)/(U_{k+P+1} - U_{k+3})
                V3<double> C3 = mk(0.0, 0.0, 0.0);
                if (P >= 3) {
#pragma unroll
                    for (int j = 0; j + 2 < P; ++j) {
                        const V3<double> T3 = ((double)(P - 2) / (Uk[P + j] - Uk[j + 2])) * (R2[j + 1] - R2[j]);
                        C3 = C3 + D3[j] * T3;
                    }
                }
                out[3] = C3;
            }
        }
    }
#undef UK
}

// Sample i of ns: parameter, span and derivatives up to order ND.
template <int P, int ND>
__device__ __forceinline__ void sample_derivs(const DCurve& c, int i, int ns, V3<double>* out)
{
    if (c.su) {   // tabulated sample parameters (arc-length sampling)
        curve_derivs<P, ND>(c, c.su[i], c.ss[i], out);
        return;
    }
    const double u = sample_param(c, i, ns);
    curve_derivs<P, ND>(c, u, sample_span(c, i, ns, u), out);
}

// Runtime degree dispatch (uniform branch) for kernels that serve curves of
// any degree.
template <int ND>
__device__ __forceinline__ void sample_derivs_any(const DCurve& c, int i, int ns, V3<double>* out)
{
    switch (c.p) {
    case 1: sample_derivs<1, ND>(c, i, ns, out); break;
    case 2: sample_derivs<2, ND>(c, i, ns, out); break;
    case 3: sample_derivs<3, ND>(c, i, ns, out); break;
    case 4: sample_derivs<4, ND>(c, i, ns, out); break;
    case 5: sample_derivs<5, ND>(c, i, ns, out); break;
    case 6: sample_derivs<6, ND>(c, i, ns, out); break;
    default: sample_derivs<7, ND>(c, i, ns, out); break;
    }
}

// ----------------------------------------------------------- frame steps

// Axis-rule unit vector: e_a with a = argmin |t[a]| (ties to the smaller
// index), projected onto the plane normal to t and normalised.
template <class F>
__device__ __forceinline__ V3<F> axis_normal(V3<F> t)
{
    const F ax = fabs(t.x), ay = fabs(t.y), az = fabs(t.z);
    int a = 0;
    F best = ax;
    if (ay < best) { a = 1; best = ay; }
    if (az < best) { a = 2; }
    const F ta = a == 0 ? t.x : (a == 1 ? t.y : t.z);
    V3<F> q = mk(-ta * t.x, -ta * t.y, -ta * t.z);
    if (a == 0) q.x += F(1); else if (a == 1) q.y += F(1); else q.z += F(1);
    const F L = sqrt(dot(q, q));
    return divs(q, L);
}

// Step rotation M_i of the double-reflection method: H1 reflects across the
// bisector plane of the chord v1 = x_{i+1} - x_i, H2 across the plane normal
// to v2 = t_{i+1} - H1 t_i; M = H2 H1.  A zero chord uses v1 = t_i.  When
// |v2|^2 <= 1e-24 the smallest rotation taking t_i to t_{i+1} is used
// (rotation by pi about the axis-rule direction for opposite tangents).
// Every case is kept as a pair of reflections, H_k x = x - b_k (v_k . x) v_k,
// applied to vectors (or matrix columns) without forming M, with no branch:
//   double reflection:  v1, b1 = 2/|v1|^2;  v2, b2 = 2/|v2|^2;
//   smallest rotation:  H(t_i + t_{i+1}) H(t_i) (two mirrors through the
//                       axis t_i x t_{i+1}, half the angle apart);
//   equal tangents:     b1 = b2 = 0 (identity);
//   opposite tangents:  H(a x t_i) H(t_i), a the axis-rule unit normal of t_i
//                       (mirrors a quarter turn apart: rotation by pi about a).
template <class F>
struct StepRot {
    V3<F> v1, v2;
    F b1, b2;
};

template <class F>
__device__ __forceinline__ StepRot<F> make_step(V3<F> v1, V3<F> ti, V3<F> tn)
{
    StepRot<F> S;
    F c1 = dot(v1, v1);
    if (c1 == F(0)) { v1 = ti; c1 = dot(v1, v1); }
    const F b1 = F(2) * recip(c1);
    const V3<F> tL = fmadd(-(b1 * dot(v1, ti)), v1, ti);
    const V3<F> v2 = tn - tL;
    const F c2 = dot(v2, v2);
    if (c2 > F(1e-24)) {
        S.v1 = v1; S.b1 = b1;
        S.v2 = v2; S.b2 = F(2) * recip(c2);
        return S;
    }
    const V3<F> k = cross(ti, tn);
    const F kk = dot(k, k), c = dot(ti, tn);
    S.v1 = ti;
    S.b1 = F(2) * recip(dot(ti, ti));
    if (kk > F(0)) {
        S.v2 = ti + tn;
    } else if (c > F(0)) {
        S.v2 = ti; S.b1 = F(0); S.b2 = F(0);
        return S;
    } else {
        S.v2 = cross(axis_normal(ti), ti);
    }
    S.b2 = F(2) * recip(dot(S.v2, S.v2));
    return S;
}

template <class F>
__device__ __forceinline__ V3<F> apply_step(const StepRot<F>& S, V3<F> x)
{
    x = fmadd(-(S.b1 * dot(S.v1, x)), S.v1, x);
    return fmadd(-(S.b2 * dot(S.v2, x)), S.v2, x);
}

// M A for the step rotation M, column by column.
template <class F>
__device__ __forceinline__ void apply_step(const StepRot<F>& S, M3<F>& A)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const V3<F> y = apply_step(S, mk(A.m[j], A.m[3 + j], A.m[6 + j]));
        A.m[j] = y.x; A.m[3 + j] = y.y; A.m[6 + j] = y.z;
    }
}

// --------------------------------------------------------- wave/block scans

// Cross-lane moves by DPP (data-parallel primitives of the GFX9 ISA: VALU
// moves, no LDS traffic).  Controls: row_shr:n = 0x110 + n (within rows of
// 16 lanes), row_bcast:15 = 0x142 (lane 15 of each row to the next row),
// row_bcast:31 = 0x143 (lane 31 to rows 2 and 3), wave_shr:1 = 0x138.  A lane
// without a source lane receives 0 (callers discard those values).
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_val(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)(b & 0xffffffffLL));
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_val(float v)
{
    return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
template <int CTRL, class F>
__device__ __forceinline__ M3<F> dpp_m3(const M3<F>& a)
{
    M3<F> r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.m[k] = dpp_val<CTRL>(a.m[k]);
    return r;
}

// Inclusive ordered product over the wave (lane 0 earliest, later factors on
// the left): products within rows of 16 lanes (shifts 1, 2, 4, 8), then row
// totals carried to rows 1 and 3, then lane 31 to the upper half.
template <class F>
__device__ __forceinline__ M3<F> wave_inclusive_product(M3<F> x)
{
    const int lane = threadIdx.x & 63, rl = lane & 15;
    M3<F> inc = x;
    { const M3<F> o = dpp_m3<0x111>(inc); if (rl >= 1) inc = mul(inc, o); }
    { const M3<F> o = dpp_m3<0x112>(inc); if (rl >= 2) inc = mul(inc, o); }
    { const M3<F> o = dpp_m3<0x114>(inc); if (rl >= 4) inc = mul(inc, o); }
    { const M3<F> o = dpp_m3<0x118>(inc); if (rl >= 8) inc = mul(inc, o); }
    { const M3<F> o = dpp_m3<0x142>(inc); if (lane & 16) inc = mul(inc, o); }
    { const M3<F> o = dpp_m3<0x143>(inc); if (lane >= 32) inc = mul(inc, o); }
    return inc;
}

// The previous lane's value (lane 0: identity).
template <class F>
__device__ __forceinline__ M3<F> wave_shift_up1(const M3<F>& a)
{
    M3<F> r = dpp_m3<0x138>(a);
    if ((threadIdx.x & 63) == 0) r = ident<F>();
    return r;
}

// Ordered product over the block, earliest element at thread 0, later
// elements multiplied on the left.  Returns thread t's exclusive prefix
// x_{t-1} ... x_0 (identity for t = 0) and the block total in `total`.
// `lds` holds kWaves matrices.  Contains __syncthreads (call from all threads).
template <class F>
__device__ M3<F> block_exclusive_product(M3<F> x, M3<F>* lds, M3<F>& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    M3<F> inc = wave_inclusive_product<F>(x);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    M3<F> wave_prefix = ident<F>();
    for (int k = 0; k < w; ++k) wave_prefix = mul(lds[k], wave_prefix);
    M3<F> tot = ident<F>();
#pragma unroll
    for (int k = 0; k < kWaves; ++k) tot = mul(lds[k], tot);
    const M3<F> exc = wave_shift_up1<F>(inc);
    total = tot;
    __syncthreads();
    return mul(exc, wave_prefix);
}

// Same exclusive product without the block total (fewer products per thread).
template <class F>
__device__ M3<F> block_exclusive_product(M3<F> x, M3<F>* lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    M3<F> inc = wave_inclusive_product<F>(x);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    M3<F> wave_prefix = ident<F>();
    for (int k = 0; k < w; ++k) wave_prefix = mul(lds[k], wave_prefix);
    const M3<F> exc = wave_shift_up1<F>(inc);
    __syncthreads();
    return mul(exc, wave_prefix);
}

// Ordered product x_{255} ... x_0 of the block (later factors on the left),
// with the same combination order as block_exclusive_product's total; the
// result is valid in wave 0 only (the other waves skip the final combine).
template <class F>
__device__ M3<F> block_product(M3<F> x, M3<F>* lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    M3<F> inc = wave_inclusive_product<F>(x);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    M3<F> tot = ident<F>();
    if (w == 0) {
#pragma unroll
        for (int k = 0; k < kWaves; ++k) tot = mul(lds[k], tot);
    }
    __syncthreads();
    return tot;
}

// Exclusive max-scan of ints over the block (identity -1); block max in `total`.
__device__ __forceinline__ int block_exclusive_max(int x, int* lds, int& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(inc, d, 64);
        if (lane >= d) inc = max(inc, o);
    }
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int wp = -1, tot = -1;
    for (int k = 0; k < kWaves; ++k) {
        if (k < w) wp = max(wp, lds[k]);
        tot = max(tot, lds[k]);
    }
    int exc = __shfl_up(inc, 1, 64);
    if (lane == 0) exc = -1;
    total = tot;
    __syncthreads();
    return max(exc, wp);
}

}  // namespace sweep

// back to the default (contraction across statements) for code that follows
#pragma clang fp contract(fast)
