// basis_ders.hpp -- B-spline basis functions and their parameter
// derivatives up to order ND on one span, in a generic scalar type, and a
// forward-mode dual number: evaluated with one knot or one weight as a dual
// variable they give the partial derivatives of C, C', C'' with respect to
// that knot or weight (the adjoint's knot and weight gradients).
#pragma once

#include <hip/hip_runtime.h>

namespace sweep {

// a + b eps with eps^2 = 0.
struct Dual {
    double v, d;
};
__host__ __device__ inline Dual dual(double v, double d = 0.0) { return Dual{v, d}; }
__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.d * b.v + a.v * b.d}; }
__host__ __device__ inline Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return Dual{q, (a.d - q * b.d) / b.v};
}
__host__ __device__ inline Dual operator*(double a, Dual b) { return Dual{a * b.v, a * b.d}; }

__host__ __device__ inline double dual_part(double) { return 0.0; }
__host__ __device__ inline double dual_part(Dual a) { return a.d; }
template <class S> __host__ __device__ inline S scalar(double v) { return S(v); }
template <> __host__ __device__ inline Dual scalar<Dual>(double v) { return Dual{v, 0.0}; }

// D[d][j] = d-th derivative of N_{s-P+j,P} at u, d = 0..ND, from the local
// knots Uk[m] = U_{s-P+1+m}, m = 0..2P-1 (span s non-empty).  Cox-de Boor
// values for degrees 0..P, then the d-th derivative from the degree P-d
// values by d rounds of the derivative rule
//   N^(r+1)_{k,q+1} = (q+1) (N^(r)_{k,q}/(U_{k+q+1}-U_k) - N^(r)_{k+1,q}/(U_{k+q+2}-U_{k+1})).
// Every denominator spans the non-empty span s.
template <int P, int ND, class S>
__host__ __device__ inline void basis_ders(const S* Uk, S u, S (&D)[ND + 1][P + 1])
{
    S B[P + 1][P + 1];
    B[0][0] = scalar<S>(1.0);
#pragma unroll
    for (int q = 1; q <= P; ++q) {
        S carry = scalar<S>(0.0);
#pragma unroll
        for (int j = 0; j < q; ++j) {
            const S lo = Uk[P - q + j], hi = Uk[P + j];
            const S tmp = B[q - 1][j] / (hi - lo);
            B[q][j] = carry + (hi - u) * tmp;
            carry = (u - lo) * tmp;
        }
        B[q][q] = carry;
    }
#pragma unroll
    for (int d = 0; d <= ND; ++d) {
        S a[P + 1];
#pragma unroll
        for (int j = 0; j <= P; ++j) a[j] = scalar<S>(0.0);
        if (d <= P) {
#pragma unroll
            for (int j = 0; j <= P - d; ++j) a[j] = B[P - d][j];
#pragma unroll
            for (int q = P - d; q < P; ++q) {
                S nb[P + 1];
#pragma unroll
                for (int j = 0; j <= q + 1; ++j) {
                    S v = scalar<S>(0.0);
                    if (j >= 1) v = v + a[j - 1] / (Uk[P - 1 + j] - Uk[P - q - 2 + j]);
                    if (j <= q) v = v - a[j] / (Uk[P + j] - Uk[P - q - 1 + j]);
                    nb[j] = (double)(q + 1) * v;
                }
#pragma unroll
                for (int j = 0; j <= q + 1; ++j) a[j] = nb[j];
            }
        }
#pragma unroll
        for (int j = 0; j <= P; ++j) D[d][j] = a[j];
    }
}

// Curve derivatives C^(d), d = 0..ND, on span s from the basis derivatives,
// the local control points Pl[j] (3 doubles each, j = 0..P) and, for a
// rational curve, the local weights wl (else nullptr):
//   C = A/W, C' = (A' - W'C)/W, C'' = (A'' - 2W'C' - W''C)/W,
//   C''' = (A''' - 3W'C'' - 3W''C' - W'''C)/W
// with A^(d) = sum_j w_j N_j^(d) P_j and W^(d) = sum_j w_j N_j^(d).
template <int P, int ND, class S>
__host__ __device__ inline void curve_ders(const S (&D)[ND + 1][P + 1], const double (*Pl)[3], const S* wl,
                                           S (&out)[ND + 1][3])
{
    S A[ND + 1][3], W[ND + 1];
#pragma unroll
    for (int d = 0; d <= ND; ++d) {
        W[d] = scalar<S>(0.0);
        A[d][0] = A[d][1] = A[d][2] = scalar<S>(0.0);
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            const S b = wl ? wl[j] * D[d][j] : D[d][j];
            W[d] = W[d] + b;
#pragma unroll
            for (int e = 0; e < 3; ++e) A[d][e] = A[d][e] + Pl[j][e] * b;
        }
    }
    if (!wl) {
#pragma unroll
        for (int d = 0; d <= ND; ++d)
#pragma unroll
            for (int e = 0; e < 3; ++e) out[d][e] = A[d][e];
        return;
    }
    // binomial coefficients of the quotient rule, up to order 3
    const double bin[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
#pragma unroll
    for (int d = 0; d <= ND; ++d) {
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            S v = A[d][e];
#pragma unroll
            for (int k = 1; k <= d; ++k) v = v - bin[d][k] * (W[k] * out[d - k][e]);
            out[d][e] = v / W[0];
        }
    }
}

}  // namespace sweep
