// Image-side helpers shared by the operator kernels: precision types, the
// per-pixel factors of S~_k (Eq. 4) and the index maps of Z (zero padding
// that places pixel N/2 at grid index 0).
#pragma once

#include "wsp_devmath.h"

namespace wsp {

namespace {

template <bool kFP64>
struct Types;
template <>
struct Types<false> {
    using R = float;
    using C = float2;
};
template <>
struct Types<true> {
    using R = double;
    using C = double2;
};

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C o;
    o.x = a.x * b.x - a.y * b.y;
    o.y = a.x * b.y + a.y * b.x;
    return o;
}

// Per-pixel factors of S~_k (Eq. 4): 1 / (g(r) n) and n - 1 at pixel (j, i),
// r = rho du cycles per cell; the stack enters only through the phase
// -wbar_k (n - 1) revolutions.
__device__ __forceinline__ void pixel_factors(int j, int i, const Geom &g, double *amp, double *nm1) {
    double l = (double)(i - g.n / 2) * g.dl;
    double m = (double)(j - g.n / 2) * g.dl;
    double rho2 = l * l + m * m;
    *nm1 = n_minus_one(rho2);
    double gv = taper_g(sqrt(rho2) * g.du, g);
    *amp = 1.0 / (gv * (1.0 + *nm1));
}

template <bool kFP64>
__device__ __forceinline__ void rev_sincos(double f, typename Types<kFP64>::R *sn,
                                           typename Types<kFP64>::R *cs) {
    if constexpr (kFP64) {
        sincospi(2.0 * f, sn, cs);
    } else {
        sincos_rev((float)f, sn, cs);
    }
}

// pixel index of grid row/column V (Z places pixel N/2 at index 0), or -1
__device__ __forceinline__ int pixel_of(int V, const Geom &g) {
    int h = g.n / 2;
    if (V < h) return V + h;
    if (V >= g.G - h) return V - g.G + h;
    return -1;
}

// column U of the padded image holding pixel column i (Z places pixel N/2 at 0)
__device__ __forceinline__ int padded_of(int i, const Geom &g) {
    int U = i - g.n / 2;
    return U < 0 ? U + g.G : U;
}

}  // namespace

}  // namespace wsp
