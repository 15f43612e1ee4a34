// Device math shared by the kernel builder and the image-domain kernels.
//
// Phase arguments (the w-chirp of Eqs. (4) and (6) and the Bessel phase
// 2 pi r q) are formed and range-reduced in FP64, in revolutions; only the
// reduced fraction in [-1/2, 1/2] is handed to FP32 polynomials.
#pragma once

#include <hip/hip_runtime.h>

#include "wsp_internal.h"
#include "wsp_tables.h"

namespace wsp {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// g(r): 2-D Fourier transform of the radial Kaiser-Bessel blob (Lewitt's pair,
// n = 2, m = 0), g(r) = 2 pi a^2 / I0(beta) * I1(z) / z with
// z^2 = beta^2 - (2 pi a r)^2.  I1(z)/z = 1/2 sum_k y^k / (k! (k+1)!),
// y = z^2 / 4, is one power series for both signs of z^2 (for z^2 < 0 it is
// J1(|z|)/|z|), summed in FP64.
__device__ __forceinline__ double taper_g(double r, const Geom &g) {
    double x = kTwoPi * g.a * r;
    double y = 0.25 * (g.beta * g.beta - x * x);
    double term = 1.0, sum = 1.0;
    for (int k = 0; k < g.taper_terms; ++k) {
        term *= y * wsp_series_r[k];
        sum += term;
    }
    return g.taper_norm * 0.5 * sum;
}

// n - 1 with n = sqrt(1 - rho^2), written as -rho^2 / (1 + n).
__device__ __forceinline__ double n_minus_one(double rho2) {
    return -rho2 / (1.0 + sqrt(1.0 - rho2));
}

// Reduce a phase given in revolutions to [-1/2, 1/2].
__device__ __forceinline__ double reduce_rev(double s) { return s - rint(s); }

// sin(2 pi f), cos(2 pi f) for |f| <= 1/2 (FP32 polynomials on an octant).
__device__ __forceinline__ void sincos_rev(float f, float *sn, float *cs) {
    float k4 = rintf(4.0f * f);
    float gg = fmaf(-0.25f, k4, f);  // |gg| <= 1/8
    float g2 = gg * gg;
    float s = wsp_sin_c[WSP_SC_N - 1];
    float c = wsp_cos_c[WSP_SC_N - 1];
#pragma unroll
    for (int i = WSP_SC_N - 2; i >= 0; --i) {
        s = fmaf(s, g2, wsp_sin_c[i]);
        c = fmaf(c, g2, wsp_cos_c[i]);
    }
    s *= gg;
    int q = ((int)k4) & 3;
    float s1 = (q & 1) ? c : s;
    float c1 = (q & 1) ? s : c;
    *sn = (q & 2) ? -s1 : s1;
    *cs = ((q + 1) & 2) ? -c1 : c1;
}

// J0(x), 0 <= x < 8: Chebyshev series in u = 2 (x/8)^2 - 1, FP64 Clenshaw.
__device__ __forceinline__ double j0_small(double x) {
    double u = fma(x * x, 1.0 / 32.0, -1.0);
    double u2 = 2.0 * u;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = WSP_J0S_N - 1; j >= 1; --j) {
        double b0 = fma(u2, b1, wsp_j0s_c[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(u, b1, wsp_j0s_c[0] - b2);
}

// Fraction of r q - 1/8 revolutions in [-1/2, 1/2]: the phase of the Hankel
// form, (x - pi/4) / (2 pi) with x = 2 pi r q.  Round-to-nearest by the
// 1.5 * 2^52 shift (|r q| < 2^51).
__device__ __forceinline__ double hankel_phase_rev(double r, double q) {
    const double kShift = 6755399441055744.0;
    double s = fma(r, q, -0.125);
    double k = (s + kShift) - kShift;
    return s - k;
}

// sin(2 pi f), cos(2 pi f) for |f| <= 1/2 in FP64 (octant polynomials).
__device__ __forceinline__ void sincos_rev64(double f, double *sn, double *cs) {
    double k4 = rint(4.0 * f);
    double gg = fma(-0.25, k4, f);  // |gg| <= 1/8
    double g2 = gg * gg;
    double s = wsp_sin_c64[WSP_SC64_N - 1];
    double c = wsp_cos_c64[WSP_SC64_N - 1];
#pragma unroll
    for (int i = WSP_SC64_N - 2; i >= 0; --i) {
        s = fma(s, g2, wsp_sin_c64[i]);
        c = fma(c, g2, wsp_cos_c64[i]);
    }
    s *= gg;
    int q = ((int)k4) & 3;
    double s1 = (q & 1) ? c : s;
    double c1 = (q & 1) ? s : c;
    *sn = (q & 2) ? -s1 : s1;
    *cs = ((q + 1) & 2) ? -c1 : c1;
}

// J0(2 pi r q) for the FP64 path: the split of j0_fp64phase, every step in
// FP64.  inv = 8 / x and amp = sqrt(2 / (pi x)) come from per-node and
// per-tap factors, as there.
__device__ __forceinline__ double j0_fp64(double r, double q, double inv, double amp) {
    double x = kTwoPi * (r * q);
    if (x < 8.0) return j0_small(x);
    double sn, cs;
    sincos_rev64(hankel_phase_rev(r, q), &sn, &cs);
    double t = inv * inv;
    double P = wsp_j0l_p64[WSP_J0L64_N - 1];
    double Q = wsp_j0l_q64[WSP_J0L64_N - 1];
#pragma unroll
    for (int i = WSP_J0L64_N - 2; i >= 0; --i) {
        P = fma(P, t, wsp_j0l_p64[i]);
        Q = fma(Q, t, wsp_j0l_q64[i]);
    }
    Q *= inv;
    return amp * (P * cs - Q * sn);
}

// J0(2 pi r q) for the FP32 path, returned in FP64 for FP64 accumulation.
//   x < 8:  Chebyshev series in FP64 (no transcendental; an FP64 FMA issues
//           at the FP32 rate on CDNA without packed math);
//   x >= 8: Hankel form sqrt(2/(pi x)) (P0 cos(x - pi/4) - Q0 sin(x - pi/4)):
//           the bracket in FP32, with the phase (x - pi/4) / (2 pi) = r q - 1/8
//           revolutions reduced in FP64, and the amplitude sqrt(2/(pi x)) in
//           FP64.  The reduced phase is split into an FP32 high part, whose
//           sine and cosine come from the hardware (arguments in revolutions,
//           |f| <= 1/2; measured within 1.3e-7 of FP64), and the FP32 rounding
//           of the rest, applied to first order (sin(a + d) = sin a + d cos a,
//           |d| < 2^-25 revolutions).
// The caller passes xf = 2 pi r q and inv = 8 / x in FP32 and amp in FP64,
// formed from per-node and per-tap factors so that no division or square
// root is needed per evaluation.  The kernel values are sums of many such
// terms that cancel (the chirp oscillates over the nodes), so the products
// and sums over the nodes are kept in FP64 by the caller.
__device__ __forceinline__ double j0_fp64phase(double r, double q, float xf, float inv, double amp) {
    if (xf < 8.0f) return j0_small(kTwoPi * (r * q));
    const double f64 = hankel_phase_rev(r, q);
    const float f = (float)f64;
    const float d = (float)(kTwoPi * (f64 - (double)f));  // radians
    const float sn0 = __builtin_amdgcn_sinf(f), cs0 = __builtin_amdgcn_cosf(f);
    const float sn = fmaf(d, cs0, sn0);
    const float cs = fmaf(-d, sn0, cs0);
    float t = inv * inv;
    float P = wsp_j0l_p[WSP_J0L_N - 1];
    float Q = wsp_j0l_q[WSP_J0L_N - 1];
#pragma unroll
    for (int i = WSP_J0L_N - 2; i >= 0; --i) {
        P = fmaf(P, t, wsp_j0l_p[i]);
        Q = fmaf(Q, t, wsp_j0l_q[i]);
    }
    Q *= inv;
    return amp * (double)(P * cs - Q * sn);
}

}  // namespace wsp
