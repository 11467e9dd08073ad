/*
 * sweep_oracle.c -- plain, sequential FP64 CPU oracle for dense swept-surface
 * evaluation (a B-spline profile S swept along a B-spline path C with a
 * rotation-minimizing moving frame).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the bench's CPU
 * baseline do.  It shares no code, header or table with the HIP path.
 *
 * The paper that frames this work (arXiv 1110.5450) defines no sweep method;
 * it only declares notation for a path C, a profile S and the Frenet vectors
 * of a curve.  Every step below therefore follows a named, published method:
 *   O1-O4  B-splines: Cox (1972) / de Boor (1972) recursion for the basis and
 *          its derivative formula; clamped ("open uniform") knots and the
 *          span rule with the end-of-domain rule of Piegl & Tiller, The NURBS
 *          Book (2nd ed.), ch. 2; uniform periodic B-splines by wrapping the
 *          control polygon.
 *   O5-O7  Rotation-minimizing frame by the double-reflection method of
 *          Wang, Juettler, Zheng & Liu, "Computation of rotation minimizing
 *          frames", ACM TOG 27(1), 2008.
 *   O8     Surface X = C(u) + [r s t] S(v) and its normal from the partial
 *          derivatives, with the derivative of the continuous RMF.
 *   O10    Central finite differences of L = sum w . X + sum g . N.
 * Where a published method leaves a choice open (degenerate tangents, the
 * initial normal, sampling, orientation) the choice is stated at the step.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fopenmp -fPIC -shared.
 * FP contraction is off so every product and sum is rounded where written.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXP 7

typedef struct {
    int n;                 /* control points; for a closed curve the m distinct ones */
    int p;                 /* degree, 1..7 */
    int closed;            /* 0 open (clamped uniform or user knots), 1 periodic uniform */
    const double *ctrl;    /* n x 3 row-major */
    const double *knots;   /* open: n+p+1 values or NULL (clamped uniform); closed: ignored */
    const double *weights; /* NULL: polynomial B-spline; else n positive weights (NURBS),
                              wrapped with the control points on a closed curve */
} or_curve;

/* ---------------------------------------------------------------- O1 knots */

int or_nbasis(int n, int p, int closed) { return closed ? n + p : n; }
int or_nknots(int n, int p, int closed) { return or_nbasis(n, p, closed) + p + 1; }

/* Open, default: U = (0^{p+1}, 1/(n-p), ..., (n-p-1)/(n-p), 1^{p+1}), interior
 * knot U_{p+k} = k/(n-p) as one correctly rounded division.
 * Open, user knots: copied.  Closed periodic: U_k = k, k = 0..m+2p, with the
 * control polygon wrapped to m+p points (Q~_k = Q_{k mod m}). */
void or_knots(int n, int p, int closed, const double *user, double *U)
{
    int nk = or_nknots(n, p, closed);
    if (closed) {
        for (int k = 0; k < nk; ++k) U[k] = (double)k;
        return;
    }
    if (user) {
        memcpy(U, user, sizeof(double) * (size_t)nk);
        return;
    }
    for (int k = 0; k < nk; ++k) {
        if (k <= p) U[k] = 0.0;
        else if (k >= n) U[k] = 1.0;
        else U[k] = (double)(k - p) / (double)(n - p);
    }
}

/* ------------------------------------------------------------- O2 samples */

/* Sample i of ns.  Open: both domain ends included,
 * u_i = a + (b - a) * (i/(ns-1)) with a = U_p, b = U_n and u_{ns-1} = b.
 * Closed: the seam is not repeated, t_j = p + (m*j)/ns. */
double or_param(int n, int p, int closed, const double *U, int i, int ns)
{
    if (closed) return (double)p + (double)((long long)n * (long long)i) / (double)ns;
    double a = U[p], b = U[n];
    if (i == ns - 1) return b;
    double f = (double)i / (double)(ns - 1);
    return a + (b - a) * f;
}

/* Span: the k in [p, nb-1] with U_k <= u < U_{k+1}; for u >= U_nb the last
 * span nb-1 (end-of-domain rule).  Plain linear search of the stored knots. */
int or_span(const double *U, int nb, int p, double u)
{
    if (u >= U[nb]) return nb - 1;
    int k = p;
    while (k + 1 < nb && U[k + 1] <= u) ++k;
    return k;
}

/* --------------------------------------------------------------- O3 basis */

/* Cox-de Boor recursion with 0/0 := 0, and its derivative form
 *   D^d N_{k,q} = q [ D^{d-1} N_{k,q-1} / (U_{k+q} - U_k)
 *                   - D^{d-1} N_{k+1,q-1} / (U_{k+q+1} - U_{k+1}) ].
 * N_{k,0} is 1 exactly for k == span (this also covers u = U_nb).
 * out[d*(p+1) + j] = D^d N_{span-p+j, p}(u), d = 0..nd, j = 0..p. */
void or_basis(const double *U, int p, int span, double u, int nd, double *out)
{
    double T[4][OR_MAXP + 1][OR_MAXP + 2];
    int lo = span - p;
    memset(T, 0, sizeof T);
    for (int j = 0; j <= p + 1; ++j) T[0][0][j] = (lo + j == span) ? 1.0 : 0.0;
    for (int q = 1; q <= p; ++q) {
        for (int j = 0; j <= p; ++j) {
            int k = lo + j;
            double d1 = U[k + q] - U[k];
            double d2 = U[k + q + 1] - U[k + 1];
            double v = 0.0;
            if (d1 != 0.0) v += (u - U[k]) / d1 * T[0][q - 1][j];
            if (d2 != 0.0) v += (U[k + q + 1] - u) / d2 * T[0][q - 1][j + 1];
            T[0][q][j] = v;
            for (int d = 1; d <= nd; ++d) {
                double w = 0.0;
                if (d1 != 0.0) w += T[d - 1][q - 1][j] / d1;
                if (d2 != 0.0) w -= T[d - 1][q - 1][j + 1] / d2;
                T[d][q][j] = (double)q * w;
            }
        }
        for (int d = 0; d <= nd; ++d) T[d][q][p + 1] = 0.0;
    }
    for (int d = 0; d <= nd; ++d)
        for (int j = 0; j <= p; ++j) out[d * (p + 1) + j] = T[d][p][j];
}

/* -------------------------------------------------------------- O4 curves */

static const double *ctrl_pt(const or_curve *c, int k)
{
    return c->ctrl + 3 * (size_t)(c->closed ? k % c->n : k);
}

static double weight_of(const or_curve *c, int k)
{
    return c->weights[c->closed ? k % c->n : k];
}

/* Rational (NURBS) curve, The NURBS Book ch. 4: in homogeneous coordinates
 * A(u) = sum_k N_{k,p}(u) w_k P_k and W(u) = sum_k N_{k,p}(u) w_k are
 * polynomial B-splines, C = A / W, and the derivatives follow from
 * A^{(d)} = sum_{i=0}^{d} binom(d, i) W^{(i)} C^{(d-i)} (Leibniz rule on
 * A = W C), solved for C^{(d)} in the order d = 0, 1, 2, 3. */
static void rational_eval(const or_curve *c, const double *B, int span, int nd, double *out)
{
    double A[4][3], W[4];
    for (int d = 0; d <= nd; ++d) {
        double a[3] = {0.0, 0.0, 0.0}, wsum = 0.0;
        for (int j = 0; j <= c->p; ++j) {
            int k = span - c->p + j;
            const double *P = ctrl_pt(c, k);
            double wk = weight_of(c, k);
            double b = B[d * (c->p + 1) + j];
            a[0] += b * (wk * P[0]);
            a[1] += b * (wk * P[1]);
            a[2] += b * (wk * P[2]);
            wsum += b * wk;
        }
        for (int e = 0; e < 3; ++e) A[d][e] = a[e];
        W[d] = wsum;
    }
    static const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    for (int d = 0; d <= nd; ++d)
        for (int e = 0; e < 3; ++e) {
            double v = A[d][e];
            for (int i = 1; i <= d; ++i)
                v -= binom[d][i] * W[i] * out[3 * (d - i) + e];
            out[3 * d + e] = v / W[0];
        }
}

/* C^{(d)}(u) = sum_k D^d N_{k,p}(u) P~_k for d = 0..nd (nd <= 3);
 * out[d*3 + c] (rational curves: see rational_eval). */
void or_curve_eval(const or_curve *c, const double *U, double u, int nd, double *out)
{
    double B[4 * (OR_MAXP + 1)];
    int nb = or_nbasis(c->n, c->p, c->closed);
    int span = or_span(U, nb, c->p, u);
    or_basis(U, c->p, span, u, nd, B);
    if (c->weights) {
        rational_eval(c, B, span, nd, out);
        return;
    }
    for (int d = 0; d <= nd; ++d) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j <= c->p; ++j) {
            const double *P = ctrl_pt(c, span - c->p + j);
            double b = B[d * (c->p + 1) + j];
            acc[0] += b * P[0];
            acc[1] += b * P[1];
            acc[2] += b * P[2];
        }
        out[3 * d + 0] = acc[0];
        out[3 * d + 1] = acc[1];
        out[3 * d + 2] = acc[2];
    }
}

/* Samples of a curve: pts/d1/d2/d3 are ns x 3 (d1, d2, d3 may be NULL). */
void or_curve_samples3(const or_curve *c, int ns, double *pts, double *d1, double *d2, double *d3)
{
    int nk = or_nknots(c->n, c->p, c->closed);
    double *U = (double *)malloc(sizeof(double) * (size_t)nk);
    or_knots(c->n, c->p, c->closed, c->knots, U);
    int nd = d3 ? 3 : (d2 ? 2 : (d1 ? 1 : 0));
    for (int i = 0; i < ns; ++i) {
        double u = or_param(c->n, c->p, c->closed, U, i, ns);
        double o[12];
        or_curve_eval(c, U, u, nd, o);
        for (int e = 0; e < 3; ++e) {
            pts[3 * i + e] = o[e];
            if (d1) d1[3 * i + e] = o[3 + e];
            if (d2) d2[3 * i + e] = o[6 + e];
            if (d3) d3[3 * i + e] = o[9 + e];
        }
    }
    free(U);
}

void or_curve_samples(const or_curve *c, int ns, double *pts, double *d1, double *d2)
{
    or_curve_samples3(c, ns, pts, d1, d2, NULL);
}

/* Parameter domain [U_p, U_nb] of a curve. */
static void domain_of(const or_curve *c, double *a, double *b)
{
    int nk = or_nknots(c->n, c->p, c->closed);
    double *U = (double *)malloc(sizeof(double) * (size_t)nk);
    or_knots(c->n, c->p, c->closed, c->knots, U);
    *a = U[c->p];
    *b = U[or_nbasis(c->n, c->p, c->closed)];
    free(U);
}

/* ------------------------------------------------------- small vector ops */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static void scale_div3(const double *a, double s, double *o) { o[0] = a[0] / s; o[1] = a[1] / s; o[2] = a[2] / s; }

/* Axis rule: e_a with a = argmin_k |v[k]| (ties to the smallest k). */
static int axis_rule(const double *v)
{
    int a = 0;
    for (int k = 1; k < 3; ++k)
        if (fabs(v[k]) < fabs(v[a])) a = k;
    return a;
}

/* normalize(w - (w.t) t) */
static void project_out(const double *w, const double *t, double *o)
{
    double d = dot3(w, t);
    double q[3] = {w[0] - d * t[0], w[1] - d * t[1], w[2] - d * t[2]};
    scale_div3(q, norm3(q), o);
}

/* Reflection across the plane through the origin normal to v:
 * H w = w - (2 (v.w)/(v.v)) v. */
static void reflect(const double *v, double c, const double *w, double *o)
{
    double f = 2.0 * dot3(v, w) / c;
    o[0] = w[0] - f * v[0];
    o[1] = w[1] - f * v[1];
    o[2] = w[2] - f * v[2];
}

/* ------------------------------------------------------- O5-O7 the frame */

/* Rotation taking t0 to t1 with the smallest angle (Rodrigues), applied to w.
 * For t1 = -t0 exactly: rotation by pi about the axis-rule direction of t0. */
static void rodrigues_apply(const double *t0, const double *t1, const double *w, double *o)
{
    double k[3];
    cross3(t0, t1, k);
    double kk = dot3(k, k);
    double c = dot3(t0, t1);
    if (kk > 0.0) {
        /* R w = c w + k x w + ((k.w)/(1+c)) k, written with (1-c)/|k|^2 = 1/(1+c) */
        double kw[3];
        cross3(k, w, kw);
        double f = (1.0 - c) / kk * dot3(k, w);
        for (int e = 0; e < 3; ++e) o[e] = c * w[e] + kw[e] + f * k[e];
    } else if (c > 0.0) {
        o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
    } else {
        double e_a[3] = {0.0, 0.0, 0.0}, a[3];
        e_a[axis_rule(t0)] = 1.0;
        project_out(e_a, t0, a);
        double f = 2.0 * dot3(a, w);          /* (2 a a^T - I) w */
        for (int e = 0; e < 3; ++e) o[e] = f * a[e] - w[e];
    }
}

/*
 * Frame along the u-samples (sample-level entry).
 *   x, d1: nu x 3 positions C(u_i) and first derivatives C'(u_i).
 *   fallback_t: unit tangent used when C'(u_0) = 0 (may be NULL -> e_z).
 *   n0: optional initial normal (NULL -> axis rule).
 *   reorth: 1 re-project r_{i+1} onto the plane normal to t_{i+1} and
 *           normalise (the defining variant); 0 keep r_{i+1} = M_i r_i raw.
 * Output R: nu x 9, row i = (r_i, s_i, t_i).
 * Returns the number of steps that took the tangent-reversal fallback.
 */
int or_frame(int nu, const double *x, const double *d1, const double *fallback_t,
             const double *n0, int reorth, double *R)
{
    int nfallback = 0;
    /* O5 tangents */
    for (int i = 0; i < nu; ++i) {
        double *t = R + 9 * (size_t)i + 6;
        double L = norm3(d1 + 3 * i);
        if (L > 0.0) {
            scale_div3(d1 + 3 * i, L, t);
        } else if (i > 0) {
            memcpy(t, R + 9 * (size_t)(i - 1) + 6, 3 * sizeof(double));
        } else if (fallback_t) {
            memcpy(t, fallback_t, 3 * sizeof(double));
        } else {
            t[0] = 0.0; t[1] = 0.0; t[2] = 1.0;
        }
    }
    /* O6 initial frame */
    {
        const double *t0 = R + 6;
        double *r0 = R + 0, *s0 = R + 3;
        int done = 0;
        if (n0) {
            double d = dot3(n0, t0);
            double q[3] = {n0[0] - d * t0[0], n0[1] - d * t0[1], n0[2] - d * t0[2]};
            double nq = norm3(q);
            if (nq > 1e-8) { scale_div3(q, nq, r0); done = 1; }
        }
        if (!done) {
            double e_a[3] = {0.0, 0.0, 0.0};
            e_a[axis_rule(t0)] = 1.0;
            project_out(e_a, t0, r0);
        }
        cross3(t0, r0, s0);
    }
    /* O7 double reflection, sequentially along u */
    for (int i = 0; i + 1 < nu; ++i) {
        const double *ri = R + 9 * (size_t)i, *ti = ri + 6;
        double *rn = R + 9 * (size_t)(i + 1), *sn = rn + 3;
        const double *tn = rn + 6;
        double v1[3] = {x[3 * (i + 1)] - x[3 * i], x[3 * (i + 1) + 1] - x[3 * i + 1],
                        x[3 * (i + 1) + 2] - x[3 * i + 2]};
        double c1 = dot3(v1, v1);
        if (c1 == 0.0) { memcpy(v1, ti, sizeof v1); c1 = dot3(v1, v1); }
        double rL[3], tL[3];
        reflect(v1, c1, ri, rL);
        reflect(v1, c1, ti, tL);
        double v2[3] = {tn[0] - tL[0], tn[1] - tL[1], tn[2] - tL[2]};
        double c2 = dot3(v2, v2);
        double r1[3];
        if (c2 <= 1e-24) {
            rodrigues_apply(ti, tn, ri, r1);
            ++nfallback;
        } else {
            reflect(v2, c2, rL, r1);
        }
        if (reorth) project_out(r1, tn, rn);
        else memcpy(rn, r1, sizeof r1);
        cross3(tn, rn, sn);
    }
    return nfallback;
}

/* --------------------------------------------------------- O8 the surface */

/*
 * Rows [row0, row1) of the surface from a frame and curve samples.
 *   x, d1, d2: path samples (nu x 3); R: frame (nu x 9);
 *   S, dS: profile samples (nv x 3);
 * Outputs (any may be NULL), all over the full grid with index
 *   c*nu*nv + i*nv + j  (pos, nrm)   and   i*nv + j  (kappa):
 *   pos = x_i + S_x r_i + S_y s_i + S_z t_i
 *   nrm = (X_v x X_u)/|X_v x X_u|, 0 when that cross product is 0 or not finite,
 *     X_v = S'_x r + S'_y s + S'_z t,
 *     X_u = (|C'| - S_x a - S_y b) t + S_z t',  a = r.C''/|C'|, b = s.C''/|C'|,
 *     t' = (C'' - (C''.t) t)/|C'|  (derivative of the continuous RMF);
 *   kappa = |X_v| (|C'| + |S_x a| + |S_y b| + |S_z|(|a| + |b|)) / |X_v x X_u|,
 *     the condition number of the normal (inf where the cross product is 0).
 * If w is given, wsum[i - row0] = sum_{c,j} w[c,i,j] * pos[c,i,j] (row partial
 * of the loss), in a fixed order.
 */
void or_surface_rows(int nu, int nv, int row0, int row1,
                     const double *x, const double *d1, const double *d2, const double *R,
                     const double *S, const double *dS,
                     double *pos, double *nrm, double *kappa,
                     const double *w, const double *g, double *wsum)
{
    size_t N = (size_t)nu * (size_t)nv;
    for (int i = row0; i < row1; ++i) {
        const double *r = R + 9 * (size_t)i, *s = r + 3, *t = r + 6;
        const double *xi = x + 3 * i, *C1 = d1 + 3 * i, *C2 = d2 + 3 * i;
        double L = norm3(C1);
        double a = 0.0, b = 0.0, tp[3] = {0.0, 0.0, 0.0};
        if (L > 0.0) {
            a = dot3(r, C2) / L;
            b = dot3(s, C2) / L;
            double ct = dot3(C2, t);
            tp[0] = (C2[0] - ct * t[0]) / L;
            tp[1] = (C2[1] - ct * t[1]) / L;
            tp[2] = (C2[2] - ct * t[2]) / L;
        }
        double acc = 0.0;
        for (int j = 0; j < nv; ++j) {
            const double *Sj = S + 3 * j, *dSj = dS + 3 * j;
            double X[3], Xu[3], Xv[3], cr[3];
            double alpha = L - Sj[0] * a - Sj[1] * b;
            for (int e = 0; e < 3; ++e) {
                X[e] = xi[e] + Sj[0] * r[e] + Sj[1] * s[e] + Sj[2] * t[e];
                Xv[e] = dSj[0] * r[e] + dSj[1] * s[e] + dSj[2] * t[e];
                Xu[e] = alpha * t[e] + Sj[2] * tp[e];
            }
            cross3(Xv, Xu, cr);
            double nn = norm3(cr);
            size_t v = (size_t)i * (size_t)nv + (size_t)j;
            if (pos)
                for (int e = 0; e < 3; ++e) pos[e * N + v] = X[e];
            int ok = nn > 0.0 && isfinite(nn);
            if (nrm)
                for (int e = 0; e < 3; ++e) nrm[e * N + v] = ok ? cr[e] / nn : 0.0;
            if (kappa) {
                double num = norm3(Xv) * (L + fabs(Sj[0] * a) + fabs(Sj[1] * b) +
                                          fabs(Sj[2]) * (fabs(a) + fabs(b)));
                kappa[v] = nn > 0.0 ? num / nn : INFINITY;
            }
            if (w)
                for (int e = 0; e < 3; ++e) acc += w[e * N + v] * X[e];
            if (g && ok)
                for (int e = 0; e < 3; ++e) acc += g[e * N + v] * (cr[e] / nn);
        }
        if (wsum) wsum[i - row0] = acc;
    }
}

/* ------------------------------------------ F4 arc-length sampling */

/* Gauss-Legendre rule with 8 nodes on [-1, 1]: nodes as the roots of the
 * Legendre polynomial P_8 (Newton's method on the three-term recurrence from
 * the Chebyshev guesses cos(pi (k - 1/4)/(8 + 1/2))), weights
 * 2 / ((1 - x^2) P_8'(x)^2). */
static void gauss_legendre8(double *x, double *w)
{
    const int n = 8;
    for (int k = 0; k < n; ++k) {
        double z = cos(M_PI * (k + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* derivative at the converged root */
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

#define OR_ARC_SUB 32   /* equal sub-intervals per knot span, 8 Gauss nodes each */

/* Sampling density at u: |C'| (arc length), plus lam |C'| kappa =
 * lam |C' x C''| / |C'|^2 (lam times the rate of turn of the tangent), so
 * that its integral is arc length + lam x turning angle. */
static double density(const or_curve *c, const double *U, double u, double lam)
{
    double o[9];
    or_curve_eval(c, U, u, lam != 0.0 ? 2 : 1, o);
    double sp = norm3(o + 3);
    if (lam == 0.0) return sp;
    double cr[3];
    cross3(o + 3, o + 6, cr);
    return sp + (sp > 0.0 ? lam * norm3(cr) / (sp * sp) : 0.0);
}

/* Integral of the density over [a, b] by the 8-point Gauss-Legendre rule. */
static double speed_gl8(const or_curve *c, const double *U, double a, double b, double lam, const double *gx,
                        const double *gw)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a), part = 0.0;
    for (int k = 0; k < 8; ++k) part += gw[k] * density(c, U, mid + half * gx[k], lam);
    return half * part;
}

/*
 * Arc-length sampling of an open curve: u_i with s(u_i) = (i/(ns-1)) s(b),
 * s(u) = integral of |C'| from the domain start a to u; u_0 = a,
 * u_{ns-1} = b.  Every non-empty knot span [U_k, U_{k+1}] is cut into
 * OR_ARC_SUB equal pieces (boundaries U_k + (U_{k+1} - U_k)(m/OR_ARC_SUB),
 * the last one U_{k+1}), each integrated by 8-point Gauss-Legendre, and the
 * piece lengths are summed in order into a cumulative table.  A target's
 * piece is the last one (in order) whose cumulative start is <= the target;
 * inside it Newton's method on s(u) - target (derivative |C'(u)|) from the
 * linear guess, kept inside the bracket (a bisection step replaces a Newton
 * step that leaves it or meets |C'| = 0), until s(u) hits the target
 * exactly, |du| <= 4 eps max(1, |u|), or 40 steps.
 * u_out: ns values; returns the total length, or -1 for a closed curve.
 * With lam > 0 the same with the density |C'| (1 + lam kappa) in place of
 * |C'| (curvature-adaptive sampling: equal steps of arc length plus lam
 * times the turning angle; lam = 0 is arc length).
 */
double or_monitor_params(const or_curve *c, int ns, double lam, double *u_out)
{
    if (c->closed) return -1.0;
    double gx[8], gw[8];
    gauss_legendre8(gx, gw);
    int nk = or_nknots(c->n, c->p, 0), nb = c->n;
    double *U = (double *)malloc(sizeof(double) * (size_t)nk);
    or_knots(c->n, c->p, 0, c->knots, U);
    int npc = (nb - c->p) * OR_ARC_SUB;                 /* pieces (empty spans give empty pieces) */
    double *lo = (double *)malloc(sizeof(double) * (size_t)npc);
    double *hi = (double *)malloc(sizeof(double) * (size_t)npc);
    double *cum = (double *)malloc(sizeof(double) * (size_t)(npc + 1));
    cum[0] = 0.0;
    for (int k = c->p, q = 0; k < nb; ++k)
        for (int m = 0; m < OR_ARC_SUB; ++m, ++q) {
            double w = U[k + 1] - U[k];
            lo[q] = U[k] + w * ((double)m / OR_ARC_SUB);
            hi[q] = m + 1 < OR_ARC_SUB ? U[k] + w * ((double)(m + 1) / OR_ARC_SUB) : U[k + 1];
            cum[q + 1] = cum[q] + (w > 0.0 ? speed_gl8(c, U, lo[q], hi[q], lam, gx, gw) : 0.0);
        }
    double total = cum[npc];
    for (int i = 0; i < ns; ++i) {
        if (i == 0) { u_out[i] = U[c->p]; continue; }
        if (i == ns - 1) { u_out[i] = U[nb]; continue; }
        double target = ((double)i / (double)(ns - 1)) * total;
        int q = 0;
        for (int r = 0; r < npc; ++r)
            if (hi[r] > lo[r] && cum[r] <= target) q = r;
        double len = cum[q + 1] - cum[q];
        double u = len > 0.0 ? lo[q] + (target - cum[q]) / len * (hi[q] - lo[q]) : lo[q];
        double blo = lo[q], bhi = hi[q];
        for (int it = 0; it < 40; ++it) {
            double f = cum[q] + speed_gl8(c, U, lo[q], u, lam, gx, gw) - target;
            if (f == 0.0) break;
            if (f > 0.0) bhi = u; else blo = u;
            double sp = density(c, U, u, lam), un;
            if (sp > 0.0) un = u - f / sp;
            else un = 0.5 * (blo + bhi);
            if (!(un >= blo && un <= bhi)) un = 0.5 * (blo + bhi);
            double du = fabs(un - u);
            u = un;
            if (du <= 4.0 * 2.220446049250313e-16 * (fabs(u) > 1.0 ? fabs(u) : 1.0)) break;
        }
        u_out[i] = u;
    }
    free(cum);
    free(hi);
    free(lo);
    free(U);
    return total;
}

double or_arclength_params(const or_curve *c, int ns, double *u_out) { return or_monitor_params(c, ns, 0.0, u_out); }

/* Curve samples at given parameters (pts/d1/d2/d3 ns x 3, d1..d3 may be NULL). */
void or_curve_samples_at(const or_curve *c, int ns, const double *u, double *pts, double *d1, double *d2,
                         double *d3)
{
    int nk = or_nknots(c->n, c->p, c->closed);
    double *U = (double *)malloc(sizeof(double) * (size_t)nk);
    or_knots(c->n, c->p, c->closed, c->knots, U);
    int nd = d3 ? 3 : (d2 ? 2 : (d1 ? 1 : 0));
    for (int i = 0; i < ns; ++i) {
        double o[12];
        or_curve_eval(c, U, u[i], nd, o);
        for (int e = 0; e < 3; ++e) {
            pts[3 * i + e] = o[e];
            if (d1) d1[3 * i + e] = o[3 + e];
            if (d2) d2[3 * i + e] = o[6 + e];
            if (d3) d3[3 * i + e] = o[9 + e];
        }
    }
    free(U);
}

/*
 * Triangle list of the n_u x n_v grid (vertex (i, j) has index i n_v + j):
 * each quad (i, j), (i+1, j), (i, j+1), (i+1, j+1), j + 1 taken modulo n_v
 * when the profile is closed, gives the triangles
 *   (i, j) (i, j+1) (i+1, j)   and   (i+1, j) (i, j+1) (i+1, j+1),
 * counter-clockwise seen from the side the normal X_v x X_u points to.
 * Quads in row-major order (i, then j); returns the triangle count.
 */
long long or_triangles(int nu, int nv, int closed_v, int *tri)
{
    int nq = closed_v ? nv : nv - 1;
    long long t = 0;
    for (int i = 0; i + 1 < nu; ++i)
        for (int j = 0; j < nq; ++j) {
            int j1 = (j + 1) % nv;
            int a = i * nv + j, b = i * nv + j1, c = (i + 1) * nv + j, d = (i + 1) * nv + j1;
            if (tri) {
                int *q = tri + 3 * t;
                q[0] = a; q[1] = b; q[2] = c;
                q[3] = c; q[4] = b; q[5] = d;
            }
            t += 2;
        }
    return t;
}

/* ------------------------------------- F2 Frenet frame and sweep laws */

/* Relative size below which C'' has no component normal to t: the Frenet
 * normal is then undefined (straight pieces, inflections). */
#define OR_FRENET_EPS 1e-8

/*
 * Frenet frame (pointwise): t as in O5 (tangents computed by or_frame's O5
 * and passed in R's third column); the principal normal
 *   n = normalize(C'' - (C''.t) t)   when |C'' - (C''.t) t| > 1e-8 |C''|,
 * else the axis-rule vector of t (O6).  r = n, s = t x n (the binormal).
 * omega_out[i] (may be NULL) = |C'| tau, the rate at which the Frenet frame
 * turns about t relative to a rotation-minimizing one, with the torsion
 *   tau = det(C', C'', C3) / |C' x C''|^2   (C3 the third derivative),
 * and 0 where the normal fell back to the axis rule.
 */
void or_frenet(int nu, const double *d1, const double *d2, const double *d3, double *R, double *omega_out)
{
    for (int i = 0; i < nu; ++i) {
        double *r = R + 9 * (size_t)i, *sv = r + 3;
        const double *t = r + 6;
        const double *C1 = d1 + 3 * i, *C2 = d2 + 3 * i, *C3 = d3 + 3 * i;
        double ct = dot3(C2, t);
        double q[3] = {C2[0] - ct * t[0], C2[1] - ct * t[1], C2[2] - ct * t[2]};
        double nq = norm3(q);
        double omega = 0.0;
        if (nq > OR_FRENET_EPS * norm3(C2)) {
            scale_div3(q, nq, r);
            double k[3];
            cross3(C1, C2, k);
            double kk = dot3(k, k);
            if (kk > 0.0) omega = norm3(C1) * (dot3(k, C3) / kk);
        } else {
            double e_a[3] = {0.0, 0.0, 0.0};
            e_a[axis_rule(t)] = 1.0;
            project_out(e_a, t, r);
        }
        cross3(t, r, sv);
        if (omega_out) omega_out[i] = omega;
    }
}

/*
 * Sweep laws along u.  A law curve L(l) (open B-spline whose control points
 * hold (sigma, theta, unused)) gives at u-sample i the scale sigma and the
 * twist angle theta (radians) of the profile: the profile point S becomes
 *   p = sigma (cos th S_x - sin th S_y, sin th S_x + cos th S_y, S_z),
 * i.e. the cross-section is rotated about t by theta and scaled by sigma.
 * The law is sampled like the path (sample i of n_u on its own domain), so
 * dl/du = (law domain length) / (path domain length).
 *
 * Rows [row0, row1) of the surface for a general frame R (nu x 9, rows r, s,
 * t) whose derivatives are taken as
 *   t' = (C'' - (C''.t) t) / |C'|,
 *   r' = -(r.t') t + omega s,   s' = -(s.t') t - omega r,
 * (omega = 0: rotation-minimizing; omega = |C'| tau: Frenet), and
 *   X   = x + p_r r + p_s s + p_t t,
 *   X_u = C' + p_r r' + p_s s' + p_t t' + p'_r r + p'_s s + p'_t t,
 *   X_v = the scaled and rotated S'(v) in the frame,
 *   N   = (X_v x X_u)/|X_v x X_u| (0 when 0 or not finite),
 * all in world coordinates.  law (nu x 4: sigma, theta, dsigma/du,
 * dtheta/du) and omega (nu) may be NULL (sigma = 1, theta = 0; omega = 0).
 * kappa = |X_v| (|C'| + |p_r||r'| + |p_s||s'| + |p_t||t'| + |p'|_1) /
 * |X_v x X_u|.
 */
void or_surface_rows_ex(int nu, int nv, int row0, int row1,
                        const double *x, const double *d1, const double *d2, const double *R,
                        const double *omega, const double *law, const double *S, const double *dS,
                        double *pos, double *nrm, double *kappa)
{
    size_t N = (size_t)nu * (size_t)nv;
    for (int i = row0; i < row1; ++i) {
        const double *r = R + 9 * (size_t)i, *s = r + 3, *t = r + 6;
        const double *xi = x + 3 * i, *C1 = d1 + 3 * i, *C2 = d2 + 3 * i;
        double L = norm3(C1);
        double tp[3] = {0.0, 0.0, 0.0}, rp[3], sp[3];
        if (L > 0.0) {
            double ct = dot3(C2, t);
            for (int e = 0; e < 3; ++e) tp[e] = (C2[e] - ct * t[e]) / L;
        }
        double om = omega ? omega[i] : 0.0;
        double rt = dot3(r, tp), st = dot3(s, tp);
        for (int e = 0; e < 3; ++e) {
            rp[e] = -rt * t[e] + om * s[e];
            sp[e] = -st * t[e] - om * r[e];
        }
        double sg = 1.0, th = 0.0, dsg = 0.0, dth = 0.0;
        if (law) { sg = law[4 * i]; th = law[4 * i + 1]; dsg = law[4 * i + 2]; dth = law[4 * i + 3]; }
        double c = cos(th), sn = sin(th);
        double nrp = norm3(rp), nsp = norm3(sp), ntp = norm3(tp);
        for (int j = 0; j < nv; ++j) {
            const double *Sj = S + 3 * j, *dSj = dS + 3 * j;
            double u0 = c * Sj[0] - sn * Sj[1], u1 = sn * Sj[0] + c * Sj[1];
            double pr = sg * u0, ps = sg * u1, pt = sg * Sj[2];
            /* d/du of sigma Rot(theta) S = sigma' Rot S + sigma theta' Rot J S, J = [[0,-1],[1,0]] */
            double dpr = dsg * u0 - sg * dth * u1;
            double dps = dsg * u1 + sg * dth * u0;
            double dpt = dsg * Sj[2];
            double qr = sg * (c * dSj[0] - sn * dSj[1]), qs = sg * (sn * dSj[0] + c * dSj[1]), qt = sg * dSj[2];
            double X[3], Xu[3], Xv[3], cr[3];
            for (int e = 0; e < 3; ++e) {
                X[e] = xi[e] + pr * r[e] + ps * s[e] + pt * t[e];
                Xv[e] = qr * r[e] + qs * s[e] + qt * t[e];
                Xu[e] = C1[e] + pr * rp[e] + ps * sp[e] + pt * tp[e] + dpr * r[e] + dps * s[e] + dpt * t[e];
            }
            cross3(Xv, Xu, cr);
            double nn = norm3(cr);
            size_t v = (size_t)i * (size_t)nv + (size_t)j;
            if (pos)
                for (int e = 0; e < 3; ++e) pos[e * N + v] = X[e];
            if (nrm) {
                int ok = nn > 0.0 && isfinite(nn);
                for (int e = 0; e < 3; ++e) nrm[e * N + v] = ok ? cr[e] / nn : 0.0;
            }
            if (kappa) {
                double num = norm3(Xv) * (L + fabs(pr) * nrp + fabs(ps) * nsp + fabs(pt) * ntp +
                                          fabs(dpr) + fabs(dps) + fabs(dpt));
                kappa[v] = nn > 0.0 ? num / nn : INFINITY;
            }
        }
    }
}

/* Law values at the nu u-samples: (sigma, theta, dsigma/du, dtheta/du). */
static void law_samples(const or_curve *law, const or_curve *path, int nu, double *out)
{
    double *v = (double *)malloc(sizeof(double) * 6 * (size_t)nu);
    or_curve_samples(law, nu, v, v + 3 * (size_t)nu, NULL);
    double la, lb, pa, pb;
    domain_of(law, &la, &lb);
    domain_of(path, &pa, &pb);
    double f = (lb - la) / (pb - pa);
    for (int i = 0; i < nu; ++i) {
        out[4 * i] = v[3 * i];
        out[4 * i + 1] = v[3 * i + 1];
        out[4 * i + 2] = v[3 * (size_t)nu + 3 * i] * f;
        out[4 * i + 3] = v[3 * (size_t)nu + 3 * i + 1] * f;
    }
    free(v);
}

/* ---------------------------------------------------- O1-O8 a whole sweep */

/* Unit direction of the first nonzero leg P_{k+1} - P_k, else e_z. */
static void first_leg(const or_curve *c, double *t)
{
    t[0] = 0.0; t[1] = 0.0; t[2] = 1.0;
    for (int k = 0; k + 1 < c->n; ++k) {
        const double *a = c->ctrl + 3 * k, *b = a + 3;
        double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double L = norm3(d);
        if (L > 0.0) { scale_div3(d, L, t); return; }
    }
}

/*
 * Whole sweep: knots, samples, frame, surface rows [row0, row1).
 * frame_out (nu x 9) and aux_out (nu x 3: |C'|, a, b) may be NULL.
 * Returns the number of tangent-reversal fallbacks, or -1 on bad input.
 * OpenMP parallelises the surface over rows (each row is independent).
 */
int or_sweep(const or_curve *path, const or_curve *prof, int nu, int nv,
             const double *n0, int reorth, int row0, int row1,
             double *pos, double *nrm, double *kappa, double *frame_out)
{
    if (nu < 2 || nv < 1 || path->closed) return -1;
    double *x = (double *)malloc(sizeof(double) * 9 * (size_t)nu);
    double *d1 = x + 3 * (size_t)nu, *d2 = x + 6 * (size_t)nu;
    double *R = frame_out ? frame_out : (double *)malloc(sizeof(double) * 9 * (size_t)nu);
    double *S = (double *)malloc(sizeof(double) * 6 * (size_t)nv);
    double *dS = S + 3 * (size_t)nv;
    or_curve_samples(path, nu, x, d1, d2);
    or_curve_samples(prof, nv, S, dS, NULL);
    double ft[3];
    first_leg(path, ft);
    int nf = or_frame(nu, x, d1, ft, n0, reorth, R);
    #pragma omp parallel for schedule(static)
    for (int i = row0; i < row1; ++i)
        or_surface_rows(nu, nv, i, i + 1, x, d1, d2, R, S, dS, pos, nrm, kappa, NULL, NULL, NULL);
    free(S);
    if (!frame_out) free(R);
    free(x);
    return nf;
}

/*
 * Whole sweep with a frame mode (0 rotation-minimizing, 1 Frenet), an
 * optional law curve (NULL: none) and the path sampled uniformly in its
 * parameter (arclength = 0) or in arc length (1; not with a law), with
 * lam > 0 curvature-adaptively (see or_monitor_params).  Same outputs as or_sweep (omega_out,
 * nu values, may be NULL); with mode 0 and no law the result equals
 * or_sweep's up to rounding (the surface derivative is then assembled in
 * world instead of frame coordinates).
 */
int or_sweep_ex(const or_curve *path, const or_curve *prof, int nu, int nv,
                const double *n0, int reorth, int mode, const or_curve *law, int arclength, double lam, int row0,
                int row1, double *pos, double *nrm, double *kappa, double *frame_out, double *omega_out)
{
    if (nu < 2 || nv < 1 || path->closed || (law && law->closed) || (law && arclength)) return -1;
    double *x = (double *)malloc(sizeof(double) * 12 * (size_t)nu);
    double *d1 = x + 3 * (size_t)nu, *d2 = x + 6 * (size_t)nu, *d3 = x + 9 * (size_t)nu;
    double *R = frame_out ? frame_out : (double *)malloc(sizeof(double) * 9 * (size_t)nu);
    double *om = omega_out ? omega_out : (double *)malloc(sizeof(double) * (size_t)nu);
    double *lw = law ? (double *)malloc(sizeof(double) * 4 * (size_t)nu) : NULL;
    double *S = (double *)malloc(sizeof(double) * 6 * (size_t)nv);
    double *dS = S + 3 * (size_t)nv;
    if (arclength) {
        double *u = (double *)malloc(sizeof(double) * (size_t)nu);
        or_monitor_params(path, nu, lam, u);
        or_curve_samples_at(path, nu, u, x, d1, d2, d3);
        free(u);
    } else {
        or_curve_samples3(path, nu, x, d1, d2, d3);
    }
    or_curve_samples(prof, nv, S, dS, NULL);
    double ft[3];
    first_leg(path, ft);
    int nf = or_frame(nu, x, d1, ft, n0, reorth, R);   /* tangents (and the RMF) */
    if (mode == 1) or_frenet(nu, d1, d2, d3, R, om);
    else for (int i = 0; i < nu; ++i) om[i] = 0.0;
    if (lw) law_samples(law, path, nu, lw);
    #pragma omp parallel for schedule(static)
    for (int i = row0; i < row1; ++i)
        or_surface_rows_ex(nu, nv, i, i + 1, x, d1, d2, R, om, lw, S, dS, pos, nrm, kappa);
    free(S);
    if (lw) free(lw);
    if (!omega_out) free(om);
    if (!frame_out) free(R);
    free(x);
    return nf;
}

/* Path samples of a sweep (x, C', C'') and the fallback tangent, for tests
 * that look at the intermediate quantities. */
void or_path_samples(const or_curve *path, int nu, double *x, double *d1, double *d2, double *ft)
{
    or_curve_samples(path, nu, x, d1, d2);
    if (ft) first_leg(path, ft);
}

/* ------------------------------------------------- O10 loss and gradient */

/* L = sum_{c,i,j} (w[c,i,j] X[c,i,j] + g[c,i,j] N[c,i,j]) over the full
 * grid, sequential; w or g may be NULL (that term is left out).  N is the
 * unit normal, 0 where it is undefined. */
double or_loss(const or_curve *path, const or_curve *prof, int nu, int nv,
               const double *n0, const double *w, const double *g)
{
    double *x = (double *)malloc(sizeof(double) * (9 * (size_t)nu + 9 * (size_t)nu + 6 * (size_t)nv + (size_t)nu));
    double *d1 = x + 3 * (size_t)nu, *d2 = x + 6 * (size_t)nu;
    double *R = x + 9 * (size_t)nu;
    double *S = R + 9 * (size_t)nu, *dS = S + 3 * (size_t)nv;
    double *rs = dS + 3 * (size_t)nv;
    or_curve_samples(path, nu, x, d1, d2);
    or_curve_samples(prof, nv, S, dS, NULL);
    double ft[3];
    first_leg(path, ft);
    or_frame(nu, x, d1, ft, n0, 1, R);
    or_surface_rows(nu, nv, 0, nu, x, d1, d2, R, S, dS, NULL, NULL, NULL, w, g, rs);
    double L = 0.0;
    for (int i = 0; i < nu; ++i) L += rs[i];
    free(x);
    return L;
}

/*
 * Central finite differences (L(th + h e_k) - L(th - h e_k)) / (2h), absolute
 * step h, over every coordinate of the path control points (gP, n_path x 3)
 * and profile control points (gQ, n_prof x 3).  Either output may be NULL to
 * skip those coordinates.  OpenMP over coordinates.
 */
void or_fd_grad(const or_curve *path, const or_curve *prof, int nu, int nv,
                const double *n0, const double *w, const double *g, double h, double *gP, double *gQ)
{
    int nP = 3 * path->n, nQ = 3 * prof->n;
    int total = (gP ? nP : 0) + (gQ ? nQ : 0);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < total; ++q) {
        int onP = gP && q < nP;
        int k = onP ? q : q - (gP ? nP : 0);
        const or_curve *base = onP ? path : prof;
        int n3 = 3 * base->n;
        double *cp = (double *)malloc(sizeof(double) * (size_t)n3);
        memcpy(cp, base->ctrl, sizeof(double) * (size_t)n3);
        or_curve c = *base;
        c.ctrl = cp;
        double th = cp[k];
        cp[k] = th + h;
        double Lp = onP ? or_loss(&c, prof, nu, nv, n0, w, g) : or_loss(path, &c, nu, nv, n0, w, g);
        cp[k] = th - h;
        double Lm = onP ? or_loss(&c, prof, nu, nv, n0, w, g) : or_loss(path, &c, nu, nv, n0, w, g);
        double g = (Lp - Lm) / (2.0 * h);
        if (onP) gP[k] = g; else gQ[k] = g;
        free(cp);
    }
}

int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
