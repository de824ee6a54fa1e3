"""Generate ``fv_coeffs.h``: the fitted coefficients used by the device math.

Run:  python gen_coeffs.py   (mpmath; about two minutes)

Two families of approximations are fitted here, from the mathematical
definitions evaluated in mpmath (no coefficients are taken from any library):

1. erfcx(z) = exp(z^2) erfc(z) on z >= -Z0 (Z0 = 1/2).  With a fixed B > Z0
   the map y = (z - B + 2 Z0)/(z + B) sends [-Z0, inf) to [-1, 1) and the
   function f(y) = (z + B) erfcx(z) is smooth and bounded on [-1, 1] (it
   tends to 1/sqrt(pi) as z -> inf).  One polynomial in y then covers the
   whole range: erfcx(z) = p(y) / (z + B).  A single branch-free expansion
   of this kind follows Shepherd & Laframboise, "Chebyshev approximation of
   (1+2x)exp(x^2)erfc x in 0 <= x < inf", Math. Comp. 36 (1981); the
   weighting (z + B) instead of (1 + 2z) lets one reciprocal serve both the
   change of variable and the final scaling, and the shifted lower end lets
   the normalised Black function take the divided difference of two erfcx
   values whose first argument may be slightly negative.  The coefficients
   are a relative-error weighted least-squares fit at Chebyshev nodes; the
   fit is checked for the value and for the derivative p'(y), since the
   evaluator uses divided differences of p.

   A second, lower-degree fit of the same form (``kErfcxLo``, relative error
   ~1e-8) serves the first Householder step of the implied-volatility
   iteration, and a third (``kErfcxG``, degree 7, ~4e-6) the boundary
   points and wing maps of its initial guess, which only has to land within
   a few percent of the root for two quartically convergent steps to reach
   binary64 precision.  A third
   (``kErfcxF32``, degree 13, value ~6e-10 and derivative ~2.4e-7 relative)
   serves the binary32 solver, where binary32 rounding dominates both.

2. The inverse standard normal CDF on (0, 1/2] (initial guess only), as one
   [3/3] rational function in the tail variable r = sqrt(-2 ln p) of the
   ratio G(r) = Phi^{-1}(p)/(r - r0), r0 = sqrt(2 ln 2) the value of r at
   p = 1/2 (where Phi^{-1} has its simple zero): G is smooth and bounded
   away from zero on the whole range and tends to -1 in the tail, so one
   branch covers p in [1e-310, 1/2] without the central/tail split of
   Wichura's AS 241 (Appl. Stat. 37, 1988), and the caller needs only
   ln p, never p itself.  Fitted by iteratively re-weighted linearised
   least squares (relative error ~2e-6, ample for a starting point that
   lands a few percent from the root).
"""
from __future__ import annotations

import os

import mpmath as mp

ERFCX_Z0 = mp.mpf("0.5")
ERFCX_B = mp.mpf("4.25")
ERFCX_DEG = 25
ERFCX_LO_B = mp.mpf("3.5")
ERFCX_LO_DEG = 12
ERFCX_F32_B = mp.mpf("3.5")
ERFCX_F32_DEG = 13
ERFCX_G_B = mp.mpf("3.0")
ERFCX_G_DEG = 7
PHI_INV_G_DEG = (3, 3)
P_MIN = mp.mpf("1e-310")


def erfcx(z):
    return mp.exp(z * z) * mp.erfc(z)


def ndtri(p):
    p = mp.mpf(p)
    if mp.mpf("1e-20") < p < 0.5:
        return -mp.sqrt(2) * mp.erfinv(1 - 2 * p)
    z = -mp.sqrt(-2 * mp.log(p))
    for _ in range(200):
        dz = (mp.ncdf(z) - p) / mp.npdf(z)
        z -= dz
        if abs(dz) < mp.mpf(10) ** (-mp.mp.dps + 5) * abs(z):
            break
    return z


def _lstsq(rows, rhs):
    m, n = len(rows), len(rows[0])
    A = mp.matrix(m, n)
    b = mp.matrix(m, 1)
    for i in range(m):
        for j in range(n):
            A[i, j] = rows[i][j]
        b[i] = rhs[i]
    Q, R = mp.qr(A)
    return mp.lu_solve(R[:n, :n], (Q.T * b)[:n, 0])


def _erfcx_z(y, B):
    return (B * (1 + y) - 2 * ERFCX_Z0) / (1 - y)


def _erfcx_f(y, B):
    z = _erfcx_z(y, B)
    return (z + B) * erfcx(z)


def fit_erfcx(B, deg):
    M = 4 * deg
    ys = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / M) for k in range(M)]
    rows, rhs = [], []
    for y in ys:
        f = _erfcx_f(y, B)
        rows.append([y ** j / f for j in range(deg + 1)])
        rhs.append(1)
    c = _lstsq(rows, rhs)
    return [c[j] for j in range(deg + 1)]


def check_erfcx(c, B, n=2000):
    """Max relative error of p and of p' (coefficients rounded to binary64)
    on a dense grid of y in (-1, 1)."""
    cd = [mp.mpf(float(v)) for v in c]
    dcd = [j * cd[j] for j in range(1, len(cd))]
    f = lambda y: _erfcx_f(y, B)
    ev, ed = mp.mpf(0), mp.mpf(0)
    for k in range(1, n):
        y = mp.cos(mp.pi * k / n)
        p = mp.polyval(cd[::-1], y)
        dp = mp.polyval(dcd[::-1], y)
        ev = max(ev, abs(p / f(y) - 1))
        ed = max(ed, abs(dp / mp.diff(f, y) - 1))
    return ev, ed


def fit_rational(ts, fs, m, n, iters=4):
    qprev = [mp.mpf(1)] * len(ts)
    for _ in range(iters):
        rows, rhs = [], []
        for t, f, qp in zip(ts, fs, qprev):
            w = 1 / (abs(f) * abs(qp))
            rows.append([t ** j * w for j in range(m + 1)] + [-f * t ** j * w for j in range(1, n + 1)])
            rhs.append(f * w)
        sol = _lstsq(rows, rhs)
        P = [sol[j] for j in range(m + 1)]
        Q = [mp.mpf(1)] + [sol[m + j] for j in range(1, n + 1)]
        qprev = [mp.fsum(cq * t ** j for j, cq in enumerate(Q)) for t in ts]
    err = max(abs(mp.fsum(cp * t ** j for j, cp in enumerate(P)) / qv / f - 1)
              for t, f, qv in zip(ts, fs, qprev))
    return P, Q, err


def fit_phi_inv(N=80, deg=PHI_INV_G_DEG):
    half = mp.mpf("0.5")
    ra = mp.sqrt(-2 * mp.log(half))  # r0: r at p = 1/2
    rb = mp.sqrt(-2 * mp.log(P_MIN))
    rs = [(ra + rb) / 2 + (rb - ra) / 2 * mp.cos(mp.pi * (k + half) / N) for k in range(N)]
    fs = []
    for r in rs:
        p = mp.exp(-r * r / 2)
        fs.append(ndtri(p) / (r - ra))
    P, Q, _ = fit_rational(rs, fs, *deg, iters=6)
    # relative error of Phi^{-1} itself on a dense grid (coefficients and r0
    # rounded to binary64)
    Pd = [mp.mpf(float(v)) for v in P]
    Qd = [mp.mpf(float(v)) for v in Q]
    r0d = mp.mpf(float(ra))
    err = mp.mpf(0)
    for k in range(1, 400):
        r = ra + (rb - ra) * mp.mpf(k) / 400
        p = mp.exp(-r * r / 2)
        g = mp.polyval(Pd[::-1], r) / mp.polyval(Qd[::-1], r)
        err = max(err, abs(g * (r - r0d) / ndtri(p) - 1))
    return P, Q, ra, err


def _arr(name, vals):
    body = ",\n".join("    %s" % mp.nstr(v, 20, min_fixed=-1, max_fixed=-1) for v in vals)
    return "constexpr double %s[%d] = {\n%s\n};\n" % (name, len(vals), body)


def main():
    mp.mp.dps = 30
    ec = fit_erfcx(ERFCX_B, ERFCX_DEG)
    eval_err, deriv_err = check_erfcx(ec, ERFCX_B)
    el = fit_erfcx(ERFCX_LO_B, ERFCX_LO_DEG)
    lo_err, lo_deriv = check_erfcx(el, ERFCX_LO_B)
    e32 = fit_erfcx(ERFCX_F32_B, ERFCX_F32_DEG)
    f32_err, f32_deriv = check_erfcx(e32, ERFCX_F32_B)
    eg = fit_erfcx(ERFCX_G_B, ERFCX_G_DEG)
    g_err, g_deriv = check_erfcx(eg, ERFCX_G_B)
    gP, gQ, gr0, gerr = fit_phi_inv()
    n3 = lambda v: mp.nstr(v, 3)
    out = [
        "// Generated by gen_coeffs.py -- do not edit by hand.\n",
        "// erfcx(z), z >= -Z0:  erfcx = p(y)/(z + B),  y = (z - B + 2 Z0)/(z + B).\n",
        "// erfcx fit max rel err %s, derivative max rel err %s\n" % (n3(eval_err), n3(deriv_err)),
        "// first-Householder-step erfcx (same form, B = kErfcxLoB): max rel err %s, derivative %s\n"
        % (n3(lo_err), n3(lo_deriv)),
        "// binary32 erfcx (same form, B = kErfcxF32B): max rel err %s, derivative %s\n"
        % (n3(f32_err), n3(f32_deriv)),
        "// initial-guess erfcx (same form, B = kErfcxGB): max rel err %s, derivative %s\n"
        % (n3(g_err), n3(g_deriv)),
        "// Inverse normal CDF on (0, 1/2]: Phi^{-1}(p) = (r - r0) P(r)/Q(r),\n",
        "// r = sqrt(-2 ln p), r0 = sqrt(2 ln 2), [3/3]; max rel err %s\n" % n3(gerr),
        "#pragma once\n\nnamespace fv {\nnamespace coef {\n\n",
        "constexpr double kErfcxZ0 = %s;\n" % mp.nstr(ERFCX_Z0, 20),
        "constexpr double kErfcxB = %s;\n" % mp.nstr(ERFCX_B, 20),
        _arr("kErfcx", ec),
        "\nconstexpr double kErfcxLoB = %s;\n" % mp.nstr(ERFCX_LO_B, 20),
        _arr("kErfcxLo", el),
        "\nconstexpr double kErfcxF32B = %s;\n" % mp.nstr(ERFCX_F32_B, 20),
        _arr("kErfcxF32", e32),
        "\nconstexpr double kErfcxGB = %s;\n" % mp.nstr(ERFCX_G_B, 20),
        _arr("kErfcxG", eg),
        "\n",
        "constexpr double kPhiInvGR0 = %s;\n" % mp.nstr(gr0, 20),
        _arr("kPhiInvGP", gP),
        _arr("kPhiInvGQ", gQ),
        "\n}  // namespace coef\n}  // namespace fv\n",
    ]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fv_coeffs.h")
    with open(path, "w") as f:
        f.write("".join(out))
    print("wrote", path, "erfcx", n3(eval_err), n3(deriv_err), "erfcx lo", n3(lo_err),
          n3(lo_deriv), "erfcx guess", n3(g_err), "phi^-1", n3(gerr))


if __name__ == "__main__":
    main()
