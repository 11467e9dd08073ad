"""Planted mistakes for the oracle's pin tests (data only).

Each entry names a plausible mistake and gives it as a text substitution on
``oracle/sweep_oracle.c``: ``original`` must occur exactly once in the clean
source, and the mutant is the source with it replaced by ``mutated``.  The
oracle source itself therefore holds only the correct formulas;
``tests/test_oracle_mutants.py`` builds every mutant with gcc and runs the pin
suite against it.
"""

MUTANTS = {
    1: ("Cox-de Boor: wrong factor (u - U_{k+1}) in the right-hand term",
        "v += (U[k + q + 1] - u) / d2", "v += (u - U[k + 1]) / d2"),
    2: ("basis derivative: the factor q dropped",
        "T[d][q][j] = (double)q * w;", "T[d][q][j] = w;"),
    3: ("sample parameter i/n_s instead of i/(n_s - 1)",
        "double f = (double)i / (double)(ns - 1);", "double f = (double)i / (double)ns;"),
    4: ("periodic wrap off by one control point",
        "(c->closed ? k % c->n : k)", "(c->closed ? (k + 1) % c->n : k)"),
    5: ("double reflection: second reflection skipped",
        "            reflect(v2, c2, rL, r1);", "            memcpy(r1, rL, sizeof r1);"),
    6: ("double reflection: chord x_{i+1} + x_i instead of the difference",
        "        double c1 = dot3(v1, v1);\n",
        "        for (int e = 0; e < 3; ++e) v1[e] = x[3 * (i + 1) + e] + x[3 * i + e];\n"
        "        double c1 = dot3(v1, v1);\n"),
    7: ("axis rule: argmax instead of argmin",
        "if (fabs(v[k]) < fabs(v[a])) a = k;", "if (fabs(v[k]) > fabs(v[a])) a = k;"),
    8: ("surface: sign of the S_x a term in X_u",
        "double alpha = L - Sj[0] * a - Sj[1] * b;", "double alpha = L + Sj[0] * a - Sj[1] * b;"),
    9: ("normal: X_u x X_v (orientation flipped)",
        "            cross3(Xv, Xu, cr);\n            double nn = norm3(cr);\n            size_t v = (size_t)i * (size_t)nv + (size_t)j;\n            if (pos)\n                for (int e = 0; e < 3; ++e) pos[e * N + v] = X[e];\n            int ok",
        "            cross3(Xu, Xv, cr);\n            double nn = norm3(cr);\n            size_t v = (size_t)i * (size_t)nv + (size_t)j;\n            if (pos)\n                for (int e = 0; e < 3; ++e) pos[e * N + v] = X[e];\n            int ok"),
    10: ("rational C'': the Leibniz factor 2 dropped",
         "v -= binom[d][i] * W[i]", "v -= (d == 2 && i == 1 ? 1.0 : binom[d][i]) * W[i]"),
    11: ("surface: the S_z t' term of X_u dropped",
         "Xu[e] = alpha * t[e] + Sj[2] * tp[e];", "Xu[e] = alpha * t[e];"),
    12: ("clamped knots k/(n-p+1)",
         "(double)(k - p) / (double)(n - p);", "(double)(k - p) / (double)(n - p + 1);"),
    13: ("frame: s = r x t (left-handed)",
         "        cross3(tn, rn, sn);", "        cross3(rn, tn, sn);"),
    14: ("finite differences divided by h instead of 2h",
         "double g = (Lp - Lm) / (2.0 * h);", "double g = (Lp - Lm) / h;"),
    15: ("frame derivative: sign of the omega term in r'",
         "rp[e] = -rt * t[e] + om * s[e];", "rp[e] = -rt * t[e] - om * s[e];"),
    16: ("twist law: sign of sigma theta' in the derivative of the profile point",
         "double dps = dsg * u1 + sg * dth * u0;", "double dps = dsg * u1 - sg * dth * u0;"),
    17: ("Frenet torsion rate doubled",
         "(dot3(k, C3) / kk);", "(dot3(k, C3) / kk) * 2.0;"),
    18: ("arc-length targets i/n_s instead of i/(n_s - 1)",
         "((double)i / (double)(ns - 1)) * total;", "((double)i / (double)ns) * total;"),
    19: ("first triangle of each quad wound clockwise",
         "q[0] = a; q[1] = b; q[2] = c;", "q[0] = a; q[1] = c; q[2] = b;"),
    20: ("normal term of the loss: the cross product not normalised",
         "acc += g[e * N + v] * (cr[e] / nn);", "acc += g[e * N + v] * cr[e];"),
    21: ("adaptive sampling density: lam |C' x C''| / |C'|^3 (kappa without |C'|)",
         "lam * norm3(cr) / (sp * sp)", "lam * norm3(cr) / (sp * sp * sp)"),
    22: ("normal condition number: the |X_v| factor dropped",
         "double num = norm3(Xv) * (L + fabs(Sj[0] * a)", "double num = (L + fabs(Sj[0] * a)"),
    23: ("normal condition number: the |S_z| (|a| + |b|) term dropped",
         "fabs(Sj[2]) * (fabs(a) + fabs(b)));", "0.0 * (fabs(a) + fabs(b)));"),
    24: ("normal condition number (frame modes, laws): the law-derivative terms dropped",
         "fabs(dpr) + fabs(dps) + fabs(dpt));", "0.0 * (fabs(dpr) + fabs(dps) + fabs(dpt)));"),
    25: ("normal condition number: |S_x a| + |S_y b| without absolute values",
         "(L + fabs(Sj[0] * a) + fabs(Sj[1] * b) +", "(L + Sj[0] * a + Sj[1] * b +"),
}


def mutate(src: str, k: int) -> str:
    """The oracle source with planted mistake k."""
    _, original, mutated = MUTANTS[k]
    n = src.count(original)
    if n != 1:
        raise ValueError(f"mutant {k}: the original text occurs {n} times in the oracle source")
    return src.replace(original, mutated)
