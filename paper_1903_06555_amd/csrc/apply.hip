// Operator application: y = Phi x (degrid) and x = Re Phi^dagger y (grid),
// Eqs. (2)-(7).  Per stack k:
//   degrid: S~_k and Z (k_taper_pad), F (hipFFT, batched over stacks),
//           GC_k and W_k (k_degrid);
//   grid:   W_k, GC_k^dagger (k_grid), F^dagger (hipFFT), Z^dagger, S~_k^dagger,
//           Re and the sum over stacks (k_crop_untaper).
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

// exp(-2 pi i wbar (n - 1)) / (g(r) n) for pixel (j, i): returns (magnitude,
// reduced phase in revolutions).  r = rho du cycles per cell.
__device__ __forceinline__ void stack_correction(int j, int i, double wbar, const Geom &g,
                                                 double *amp, double *rev) {
    double l = (double)(i - g.n / 2) * g.dl;
    double m = (double)(j - g.n / 2) * g.dl;
    double rho2 = l * l + m * m;
    double nm1 = n_minus_one(rho2);
    double n = 1.0 + nm1;
    double gv = taper_g(sqrt(rho2) * g.du, g);
    *amp = 1.0 / (gv * n);
    *rev = reduce_rev(-wbar * nm1);
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

template <bool kFP64>
__global__ void k_taper_pad(const typename Types<kFP64>::R *__restrict__ image,
                            typename Types<kFP64>::C *grids, const double *__restrict__ centres,
                            Geom g) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const int64_t GG = (int64_t)g.G * g.G;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= GG * g.n_stacks) return;
    int k = (int)(idx / GG);
    int64_t cell = idx - (int64_t)k * GG;
    int V = (int)(cell / g.G), U = (int)(cell - (int64_t)V * g.G);
    int j = pixel_of(V, g), i = pixel_of(U, g);
    C z;
    z.x = 0;
    z.y = 0;
    if (j >= 0 && i >= 0) {
        double amp, rev;
        stack_correction(j, i, centres[k], g, &amp, &rev);
        R sn, cs;
        rev_sincos<kFP64>(rev, &sn, &cs);
        R a = (R)((double)image[(int64_t)j * g.n + i] * amp);
        z.x = a * cs;
        z.y = a * sn;
    }
    grids[idx] = z;
}

template <bool kFP64>
__global__ void k_crop_untaper(const typename Types<kFP64>::C *__restrict__ grids,
                               typename Types<kFP64>::R *image, const double *__restrict__ centres,
                               Geom g) {
    using R = typename Types<kFP64>::R;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)g.n * g.n) return;
    int j = (int)(idx / g.n), i = (int)(idx - (int64_t)j * g.n);
    int V = (j - g.n / 2 + g.G) % g.G, U = (i - g.n / 2 + g.G) % g.G;
    const int64_t GG = (int64_t)g.G * g.G;
    double acc = 0.0;
    for (int k = 0; k < g.n_stacks; ++k) {
        double amp, rev;
        stack_correction(j, i, centres[k], g, &amp, &rev);
        R sn, cs;
        rev_sincos<kFP64>(rev, &sn, &cs);
        auto z = grids[k * GG + (int64_t)V * g.G + U];
        // Re(z conj(s_k)) with s_k = amp e^{2 pi i rev}
        acc += amp * (double)(z.x * cs + z.y * sn);
    }
    image[idx] = (R)acc;
}

template <typename C>
__global__ void k_zero(C *x, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        C z;
        z.x = 0;
        z.y = 0;
        x[i] = z;
    }
}

struct ApplyArgs {
    const int32_t *perm, *jp, *u0w, *v0w, *stack;
    const double *wt;
    const uint8_t *sflag;
    const int64_t *tap_off;
    int64_t m;
    Geom g;
};

__device__ __forceinline__ int wrap_index(int x, int G) {
    while (x >= G) x -= G;
    return x;
}

template <typename R>
__device__ __forceinline__ R wave_sum_r(R x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// GC_k, W_k: one wavefront per visibility (sorted order), lanes over taps.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_degrid(const typename Types<kFP64>::C *__restrict__ taps,
                                                const typename Types<kFP64>::C *__restrict__ grids,
                                                typename Types<kFP64>::C *vis, ApplyArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const int lane = threadIdx.x & 63;
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.m) return;
    const int G = a.g.G;
    const int jp = a.jp[p];
    const int u0 = a.u0w[p], v0 = a.v0w[p];
    const C *tp = taps + a.tap_off[p];
    const C *gk = grids + (int64_t)a.stack[p] * G * G;
    const int ntap = jp * jp;
    R ar = 0, ai = 0;
    for (int t = lane; t < ntap; t += 64) {
        int row = t / jp, col = t - row * jp;
        int V = wrap_index(v0 + row, G), U = wrap_index(u0 + col, G);
        C K = tp[t];
        C z = gk[(int64_t)V * G + U];
        ar += K.x * z.x - K.y * z.y;
        ai += K.x * z.y + K.y * z.x;
    }
    ar = wave_sum_r(ar);
    ai = wave_sum_r(ai);
    if (lane == 0) {
        R w = (R)a.wt[p];
        C y;
        y.x = ar * w;
        y.y = (a.sflag[p] ? -ai : ai) * w;  // Eq. (8): folded visibilities are conjugated
        vis[a.perm[p]] = y;
    }
}

// GC_k^dagger, W_k: one wavefront per visibility, conj(K) y added with atomics.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_grid(const typename Types<kFP64>::C *__restrict__ taps,
                                              const typename Types<kFP64>::C *__restrict__ vis,
                                              typename Types<kFP64>::C *grids, ApplyArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const int lane = threadIdx.x & 63;
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.m) return;
    const int G = a.g.G;
    const int jp = a.jp[p];
    const int u0 = a.u0w[p], v0 = a.v0w[p];
    const C *tp = taps + a.tap_off[p];
    C *gk = grids + (int64_t)a.stack[p] * G * G;
    C y = vis[a.perm[p]];
    R w = (R)a.wt[p];
    R yr = y.x * w, yi = (a.sflag[p] ? -y.y : y.y) * w;
    const int ntap = jp * jp;
    for (int t = lane; t < ntap; t += 64) {
        int row = t / jp, col = t - row * jp;
        int V = wrap_index(v0 + row, G), U = wrap_index(u0 + col, G);
        C K = tp[t];
        R *dst = (R *)(gk + (int64_t)V * G + U);
        atomicAdd(dst, K.x * yr + K.y * yi);
        atomicAdd(dst + 1, K.x * yi - K.y * yr);
    }
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

ApplyArgs make_args(const wsp_ctx *c) {
    const Plan &pl = c->plan;
    ApplyArgs a{};
    a.perm = pl.perm;
    a.jp = pl.jp;
    a.u0w = pl.u0w;
    a.v0w = pl.v0w;
    a.stack = pl.stack;
    a.wt = pl.wt;
    a.sflag = pl.sflag;
    a.tap_off = pl.tap_off;
    a.m = pl.m;
    a.g = c->g;
    return a;
}

hipError_t fft_exec(wsp_ctx *c, bool forward, hipStream_t s) {
    if (hipfftSetStream(c->fft, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
    hipfftResult r;
    if (c->p.precision == WSP_FP64) {
        r = hipfftExecZ2Z(c->fft, (hipfftDoubleComplex *)c->grids, (hipfftDoubleComplex *)c->grids,
                          forward ? HIPFFT_FORWARD : HIPFFT_BACKWARD);
    } else {
        r = hipfftExecC2C(c->fft, (hipfftComplex *)c->grids, (hipfftComplex *)c->grids,
                          forward ? HIPFFT_FORWARD : HIPFFT_BACKWARD);
    }
    return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown;
}

template <bool kFP64>
hipError_t degrid_t(wsp_ctx *c, const void *image, void *vis, const double *d_centres,
                    hipStream_t s) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const Geom &g = c->g;
    int64_t ncell = (int64_t)g.G * g.G * g.n_stacks;
    hipEvent_t ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_taper_pad<kFP64>, dim3(blocks(ncell, 256)), dim3(256), 0, s,
                       (const R *)image, (C *)c->grids, d_centres, g);
    stage_end(c, kStTaperPad, ev, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ev = stage_begin(c, s);
    e = fft_exec(c, true, s);
    stage_end(c, kStFftForward, ev, s);
    if (e != hipSuccess) return e;
    ApplyArgs a = make_args(c);
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_degrid<kFP64>, dim3(blocks(a.m * 64, 256)), dim3(256), 0, s,
                       (const C *)c->taps, (const C *)c->grids, (C *)vis, a);
    stage_end(c, kStDegrid, ev, s);
    return hipGetLastError();
}

template <bool kFP64>
hipError_t grid_t(wsp_ctx *c, const void *vis, void *image, const double *d_centres,
                  hipStream_t s) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const Geom &g = c->g;
    int64_t ncell = (int64_t)g.G * g.G * g.n_stacks;
    hipEvent_t ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_zero<C>, dim3(blocks(ncell, 256)), dim3(256), 0, s, (C *)c->grids, ncell);
    stage_end(c, kStZero, ev, s);
    ApplyArgs a = make_args(c);
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_grid<kFP64>, dim3(blocks(a.m * 64, 256)), dim3(256), 0, s,
                       (const C *)c->taps, (const C *)vis, (C *)c->grids, a);
    stage_end(c, kStGrid, ev, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ev = stage_begin(c, s);
    e = fft_exec(c, false, s);
    stage_end(c, kStFftInverse, ev, s);
    if (e != hipSuccess) return e;
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_crop_untaper<kFP64>, dim3(blocks((int64_t)g.n * g.n, 256)), dim3(256), 0,
                       s, (const C *)c->grids, (R *)image, d_centres, g);
    stage_end(c, kStCropUntaper, ev, s);
    return hipGetLastError();
}

}  // namespace

hipError_t run_degrid(wsp_ctx *c, const void *image, void *vis, hipStream_t s) {
    if (c->p.precision == WSP_FP64) return degrid_t<true>(c, image, vis, c->plan_centres, s);
    return degrid_t<false>(c, image, vis, c->plan_centres, s);
}

hipError_t run_grid(wsp_ctx *c, const void *vis, void *image, hipStream_t s) {
    if (c->p.precision == WSP_FP64) return grid_t<true>(c, vis, image, c->plan_centres, s);
    return grid_t<false>(c, vis, image, c->plan_centres, s);
}

}  // namespace wsp
