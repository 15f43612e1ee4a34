"""Generate wsp_tables.h: quadrature rule and FP32 polynomial fits for the HIP builder.

Run from the repository root:  python paper_1903_06555_amd/csrc/gen_tables.py

Everything is derived here from its mathematical definition with mpmath at
50 digits; nothing is copied from a math library:

- Gauss-Kronrod (7, 15) rule on [-1, 1]: Gauss-Legendre nodes from the roots
  of P_7, Kronrod nodes from the roots of the Stieltjes polynomial E_8
  (orthogonal to x^k P_7(x), k = 0..7; Kronrod 1965), weights from exactness
  on monomials up to degree 14 (checked to degree 22 = 3n + 1);
- J0 on [0, 8]: Chebyshev interpolant in u = 2 (x/8)^2 - 1 (J0 is even in x),
  evaluated in FP64 by the builder (FP32 Clenshaw would lose ~10 ulp);
- J0 for x >= 8 through the Hankel form
  J0(x) = sqrt(2 / (pi x)) (P0 cos(x - pi/4) - Q0 sin(x - pi/4)),
  with P0 and x Q0 / 8 fitted as polynomials in t = (8/x)^2 on (0, 1]; exact
  P0, Q0 come from J0 and Y0 (Abramowitz & Stegun 9.2.5);
- sin(2 pi g), cos(2 pi g) on |g| <= 1/8 (revolutions) as odd/even polynomials.
"""
from __future__ import annotations

import os

import mpmath as mp

mp.mp.dps = 50

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wsp_tables.h")


def legendre_poly_coeffs(n):
    # monomial coefficients (ascending) of P_n via the three-term recurrence
    p0, p1 = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    if n == 0:
        return p0
    for k in range(1, n):
        nxt = [mp.mpf(0)] * (k + 2)
        for i, c in enumerate(p1):
            nxt[i + 1] += (2 * k + 1) * c / (k + 1)
        for i, c in enumerate(p0):
            nxt[i] -= k * c / (k + 1)
        p0, p1 = p1, nxt
    return p1


def integrate_monomial(k):
    return mp.mpf(0) if k % 2 else mp.mpf(2) / (k + 1)


def poly_mul(a, b):
    out = [mp.mpf(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def gauss_kronrod(n):
    Pn = legendre_poly_coeffs(n)
    gauss = sorted(mp.polyroots(list(reversed(Pn)), maxsteps=200, extraprec=200))
    gauss = [mp.re(g) for g in gauss]
    # Stieltjes polynomial E_{n+1} = x^{n+1} + sum_{j<=n} c_j x^j, orthogonal to x^k P_n
    m = n + 1
    A = mp.matrix(n + 1, n + 1)
    rhs = mp.matrix(n + 1, 1)
    for k in range(n + 1):
        base = poly_mul(Pn, [mp.mpf(0)] * k + [mp.mpf(1)])
        mom = lambda j: sum(c * integrate_monomial(i + j) for i, c in enumerate(base))
        for j in range(n + 1):
            A[k, j] = mom(j)
        rhs[k] = -mom(m)
    c = mp.lu_solve(A, rhs)
    E = [c[j] for j in range(n + 1)] + [mp.mpf(1)]
    kron = [mp.re(r) for r in mp.polyroots(list(reversed(E)), maxsteps=400, extraprec=400)]
    nodes = sorted(gauss + kron)
    N = len(nodes)
    V = mp.matrix(N, N)
    b = mp.matrix(N, 1)
    for k in range(N):
        for j, x in enumerate(nodes):
            V[k, j] = x ** k
        b[k] = integrate_monomial(k)
    w = mp.lu_solve(V, b)
    wk = [w[j] for j in range(N)]
    for k in range(3 * n + 2):
        err = sum(wk[j] * nodes[j] ** k for j in range(N)) - integrate_monomial(k)
        assert abs(err) < mp.mpf(10) ** -40, (k, err)
    # Gauss weights
    Vg = mp.matrix(n, n)
    bg = mp.matrix(n, 1)
    for k in range(n):
        for j, x in enumerate(gauss):
            Vg[k, j] = x ** k
        bg[k] = integrate_monomial(k)
    wg = mp.lu_solve(Vg, bg)
    wgauss = []
    for x in nodes:
        idx = [i for i, g in enumerate(gauss) if abs(g - x) < mp.mpf(10) ** -40]
        wgauss.append(wg[idx[0]] if idx else mp.mpf(0))
    return nodes, wk, wgauss


def chebyshev_fit(f, deg):
    # interpolate f(u) on [-1, 1] at Chebyshev nodes, return Chebyshev coefficients
    N = deg + 1
    us = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / N) for k in range(N)]
    fs = [f(u) for u in us]
    coeffs = []
    for j in range(N):
        s = sum(fs[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / N) for k in range(N))
        coeffs.append(2 * s / N if j else s / N)
    return coeffs


def cheb_to_monomial(c):
    # coefficients of sum c_j T_j(u) in powers of u
    T_prev, T_cur = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    out = [mp.mpf(0)] * len(c)
    out[0] += c[0]
    if len(c) > 1:
        out[1] += c[1]
    for j in range(2, len(c)):
        T_next = [mp.mpf(0)] * (j + 1)
        for i, v in enumerate(T_cur):
            T_next[i + 1] += 2 * v
        for i, v in enumerate(T_prev):
            T_next[i] -= v
        for i, v in enumerate(T_next):
            out[i] += c[j] * v
        T_prev, T_cur = T_cur, T_next
    return out


def fit_in_t(f, deg, t0, t1):
    # polynomial in t on [t0, t1] via Chebyshev interpolation, returned in powers of t
    mid, half = (t0 + t1) / 2, (t1 - t0) / 2
    c = chebyshev_fit(lambda u: f(mid + half * u), deg)
    mono_u = cheb_to_monomial(c)
    # substitute u = (t - mid) / half
    out = [mp.mpf(0)] * len(mono_u)
    for k, a in enumerate(mono_u):
        # (t - mid)^k / half^k
        for i in range(k + 1):
            out[i] += a * mp.binomial(k, i) * (-mid) ** (k - i) / half ** k
    return out


def max_err(f, approx, a, b, n=4000):
    return max(abs(f(a + (b - a) * mp.mpf(i) / n) - approx(a + (b - a) * mp.mpf(i) / n))
               for i in range(n + 1))


def horner(coeffs, t):
    acc = mp.mpf(0)
    for c in reversed(coeffs):
        acc = acc * t + c
    return acc


def clenshaw(c, u):
    b1 = b2 = mp.mpf(0)
    for cj in reversed(c[1:]):
        b1, b2 = 2 * u * b1 - b2 + cj, b1
    return u * b1 - b2 + c[0]


def main():
    lines = ["/* Generated by gen_tables.py -- do not edit. */",
             "#pragma once", "", "#include <hip/hip_runtime.h>", ""]
    nodes, wk, wg = gauss_kronrod(7)
    lines.append("/* Gauss-Kronrod (7, 15) on [-1, 1]: nodes, Kronrod weights, Gauss weights (0 off-Gauss). */")
    lines.append("#define WSP_GK_N 15")
    for name, arr in (("wsp_gk_x", nodes), ("wsp_gk_wk", wk), ("wsp_gk_wg", wg)):
        lines.append(f"static __constant__ double {name}[15] = {{" +
                     ", ".join(mp.nstr(v, 20, min_fixed=-1, max_fixed=1) for v in arr) + "};")

    # J0 on [0, 8] in u = 2 (x/8)^2 - 1
    deg_small = 16
    f_small = lambda u: mp.besselj(0, 8 * mp.sqrt((u + 1) / 2))
    cs = chebyshev_fit(f_small, deg_small)
    err_s = max_err(f_small, lambda u: clenshaw(cs, u), -1, 1)
    lines.append(f"/* J0(x), 0 <= x < 8: sum_j c_j T_j(u), u = 2 (x/8)^2 - 1; max interp error {mp.nstr(err_s, 3)} */")
    lines.append(f"#define WSP_J0S_N {deg_small + 1}")
    lines.append("static __constant__ double wsp_j0s_c[] = {" + ", ".join(mp.nstr(v, 20) for v in cs) + "};")

    # Hankel form for x >= 8, t = (8/x)^2 in (0, 1]
    def p0q0(x):
        chi = x - mp.pi / 4
        s = mp.sqrt(mp.pi * x / 2)
        J, Y = mp.besselj(0, x), mp.bessely(0, x)
        return s * (J * mp.cos(chi) + Y * mp.sin(chi)), s * (-J * mp.sin(chi) + Y * mp.cos(chi))
    tmin = mp.mpf(1) / 10 ** 6
    fP = lambda t: p0q0(8 / mp.sqrt(t))[0]
    fR = lambda t: p0q0(8 / mp.sqrt(t))[1] * (8 / mp.sqrt(t)) / 8
    deg_l = 3
    cP = fit_in_t(fP, deg_l, tmin, mp.mpf(1))
    cR = fit_in_t(fR, deg_l, tmin, mp.mpf(1))
    eP = max_err(fP, lambda t: horner(cP, t), tmin, 1)
    eR = max_err(fR, lambda t: horner(cR, t), tmin, 1)
    lines.append(f"/* x >= 8, t = (8/x)^2: P0 = sum p_k t^k (err {mp.nstr(eP, 3)}), Q0 = (8/x) sum q_k t^k (err {mp.nstr(eR, 3)}) */")
    lines.append(f"#define WSP_J0L_N {deg_l + 1}")
    lines.append("static __constant__ float wsp_j0l_p[] = {" + ", ".join(mp.nstr(v, 12) + "f" for v in cP) + "};")
    lines.append("static __constant__ float wsp_j0l_q[] = {" + ", ".join(mp.nstr(v, 12) + "f" for v in cR) + "};")

    # sin(2 pi g) = g * S(g^2), cos(2 pi g) = C(g^2), |g| <= 1/8
    gmax2 = mp.mpf(1) / 64
    fS = lambda s: (mp.sin(2 * mp.pi * mp.sqrt(s)) / mp.sqrt(s)) if s > 0 else 2 * mp.pi
    fC = lambda s: mp.cos(2 * mp.pi * mp.sqrt(s))
    cS = fit_in_t(fS, 4, mp.mpf(0), gmax2)
    cC = fit_in_t(fC, 4, mp.mpf(0), gmax2)
    eS = max_err(lambda g: mp.sin(2 * mp.pi * g), lambda g: g * horner(cS, g * g), 0, mp.mpf(1) / 8)
    eC = max_err(lambda g: mp.cos(2 * mp.pi * g), lambda g: horner(cC, g * g), 0, mp.mpf(1) / 8)
    lines.append(f"/* sin(2 pi g) = g sum s_k g^2k (err {mp.nstr(eS, 3)}), cos(2 pi g) = sum c_k g^2k (err {mp.nstr(eC, 3)}), |g| <= 1/8 */")
    lines.append("#define WSP_SC_N 5")
    lines.append("static __constant__ float wsp_sin_c[] = {" + ", ".join(mp.nstr(v, 12) + "f" for v in cS) + "};")
    lines.append("static __constant__ float wsp_cos_c[] = {" + ", ".join(mp.nstr(v, 12) + "f" for v in cC) + "};")
    # FP64 path: the same Hankel form and octant sine / cosine, fitted to FP64 accuracy
    deg_l64 = 8
    cP64 = fit_in_t(fP, deg_l64, tmin, mp.mpf(1))
    cR64 = fit_in_t(fR, deg_l64, tmin, mp.mpf(1))
    eP64 = max_err(fP, lambda t: horner(cP64, t), tmin, 1)
    eR64 = max_err(fR, lambda t: horner(cR64, t), tmin, 1)
    lines.append(f"/* FP64 path, x >= 8: P0 (err {mp.nstr(eP64, 3)}), Q0 / (8/x) (err {mp.nstr(eR64, 3)}), powers of t = (8/x)^2 */")
    lines.append(f"#define WSP_J0L64_N {deg_l64 + 1}")
    lines.append("static __constant__ double wsp_j0l_p64[] = {" + ", ".join(mp.nstr(v, 20) for v in cP64) + "};")
    lines.append("static __constant__ double wsp_j0l_q64[] = {" + ", ".join(mp.nstr(v, 20) for v in cR64) + "};")
    deg_sc64 = 6
    cS64 = fit_in_t(fS, deg_sc64, mp.mpf(0), gmax2)
    cC64 = fit_in_t(fC, deg_sc64, mp.mpf(0), gmax2)
    eS64 = max_err(lambda g: mp.sin(2 * mp.pi * g), lambda g: g * horner(cS64, g * g), 0, mp.mpf(1) / 8)
    eC64 = max_err(lambda g: mp.cos(2 * mp.pi * g), lambda g: horner(cC64, g * g), 0, mp.mpf(1) / 8)
    lines.append(f"/* FP64 path: sin(2 pi g) = g sum s_k g^2k (err {mp.nstr(eS64, 3)}), cos(2 pi g) = sum c_k g^2k (err {mp.nstr(eC64, 3)}), |g| <= 1/8 */")
    lines.append(f"#define WSP_SC64_N {deg_sc64 + 1}")
    lines.append("static __constant__ double wsp_sin_c64[] = {" + ", ".join(mp.nstr(v, 20) for v in cS64) + "};")
    lines.append("static __constant__ double wsp_cos_c64[] = {" + ", ".join(mp.nstr(v, 20) for v in cC64) + "};")
    # Lagrange interpolation on the 10 equispaced nodes 0..9:
    # l_k(u) = c_k prod_{j != k} (u - j), c_k = (-1)^(9 - k) / (k! (9 - k)!)
    lines.append("/* 10-point equispaced Lagrange basis: c_k = (-1)^(9-k) / (k! (9-k)!) */")
    lines.append("static __constant__ double wsp_lagrange10_c[10] = {" + ", ".join(
        repr(float(mp.mpf((-1) ** (9 - k)) / (mp.factorial(k) * mp.factorial(9 - k)))) for k in range(10)) + "};")
    # reciprocals 1 / ((k + 1) (k + 2)) for the power series of I1(z) / z in z^2 / 4
    lines.append("/* 1 / ((k + 1) (k + 2)), k = 0..127: ratio of successive terms of sum_k y^k / (k! (k+1)!) */")
    lines.append("#define WSP_SERIES_N 128")
    lines.append("static __constant__ double wsp_series_r[128] = {" +
                 ", ".join(repr(1.0 / ((k + 1.0) * (k + 2.0))) for k in range(128)) + "};")
    lines.append("")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
