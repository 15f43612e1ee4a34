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

// GC_k, W_k: one wavefront per visibility, lanes over taps.  Waves are
// mapped XCD-aware: each of the 8 XCDs takes a contiguous run of the sorted
// visibilities, so the grid region it gathers from stays in its own L2.  Tap
// coordinates advance incrementally (no division in the loop).
template <bool kFP64>
__global__ __launch_bounds__(256) void k_degrid(const typename Types<kFP64>::C *__restrict__ taps,
                                                const typename Types<kFP64>::C *__restrict__ grids,
                                                typename Types<kFP64>::C *vis, ApplyArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int kU = 4;  // taps per lane in flight
    const int lane = threadIdx.x & 63;
    const int nblk = gridDim.x;
    const int per = nblk / 8;  // gridDim.x is a multiple of 8
    const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
    // wave-uniform visibility index (metadata through the scalar cache)
    const int64_t p = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
    if (p >= a.m) return;
    const int G = a.g.G;
    const int jp = a.jp[p];
    const int u0 = a.u0w[p], v0 = a.v0w[p];
    const C *tp = taps + a.tap_off[p];
    const C *gk = grids + (int64_t)a.stack[p] * G * G;
    const int ntap = jp * jp;
    // lane's first tap (t = lane) and the per-step advance of 64 taps
    int row = lane / jp, col = lane - (lane / jp) * jp;
    const int drow = 64 / jp, dcol = 64 - (64 / jp) * jp;
    int V = v0 + row;
    while (V >= G) V -= G;
    R ar = 0, ai = 0;
    for (int t0 = 0; t0 < ntap; t0 += 64 * kU) {
        C K[kU], z[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int t = t0 + 64 * u + lane;
            int U = u0 + col;
            while (U >= G) U -= G;
            if (t < ntap) {
                K[u] = tp[t];
                z[u] = gk[(int64_t)V * G + U];
            } else {
                K[u].x = K[u].y = 0;
                z[u].x = z[u].y = 0;
            }
            col += dcol;
            int dr = drow;
            if (col >= jp) {
                col -= jp;
                ++dr;
            }
            V += dr;
            while (V >= G) V -= G;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            ar += K[u].x * z[u].x - K[u].y * z[u].y;
            ai += K[u].x * z[u].y + K[u].y * z[u].x;
        }
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

// W_k and Eq. (8) on the adjoint's input: yw[p] = W_p (conj) y[perm[p]] in
// sorted order.
template <bool kFP64>
__global__ void k_prep_vis(const typename Types<kFP64>::C *__restrict__ vis,
                           typename Types<kFP64>::C *yw, ApplyArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.m) return;
    C y = vis[a.perm[p]];
    R w = (R)a.wt[p];
    C o;
    o.x = y.x * w;
    o.y = (a.sflag[p] ? -y.y : y.y) * w;
    yw[p] = o;
}

struct TileArgs {
    const int4 *ent;
    const int32_t *ent_sorted;
    const int32_t *item_start;
    const uint32_t *item_key;
    const uint8_t *item_sole;
    const int32_t *item_slot;
    void *partial;
    const int32_t *jp;
    const int64_t *tap_off;
    int n_items;
    int tile_bits;
    int G;
};

// XCD-aware block order: consecutive items (neighbouring tiles) go to the
// same XCD, which dispatches blocks round-robin over its 8 dies.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int nx = 8;
    int per = (n + nx - 1) / nx;
    return (b % nx) * per + b / nx;
}

// GC_k^dagger: one block per work item (a run of entries of one grid tile).
// The tile is privatised in LDS; the four wavefronts take entries in turn,
// lanes walk the entry's tap sub-block and add conj(K) yw with LDS atomics;
// the tile is then stored (its only item) or added atomically to the grid.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_grid_tiles(const typename Types<kFP64>::C *__restrict__ taps,
                                                    const typename Types<kFP64>::C *__restrict__ yw,
                                                    typename Types<kFP64>::C *grids, TileArgs t) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int kChunk = 256;  // entries whose metadata is staged in LDS at a time
    constexpr int kU = 8;        // taps per lane in flight
    __shared__ R tre[kTile * kTile];
    __shared__ R tim[kTile * kTile];
    __shared__ int4 s_ent[kChunk];
    __shared__ int64_t s_off[kChunk];
    __shared__ int s_jp[kChunk];
    __shared__ C s_y[kChunk];
    const int item = xcd_item(blockIdx.x, t.n_items);
    if (item >= t.n_items) return;  // uniform over the block
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
        tre[i] = 0;
        tim[i] = 0;
    }
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int s_beg = t.item_start[item], s_end = t.item_start[item + 1];
    for (int base = s_beg; base < s_end; base += kChunk) {
        const int n = (s_end - base < kChunk) ? s_end - base : kChunk;
        __syncthreads();  // LDS tile cleared / previous chunk consumed
        if ((int)threadIdx.x < n) {
            const int4 en = t.ent[t.ent_sorted[base + threadIdx.x]];
            s_ent[threadIdx.x] = en;
            s_off[threadIdx.x] = t.tap_off[en.x];
            s_jp[threadIdx.x] = t.jp[en.x];
            s_y[threadIdx.x] = yw[en.x];
        }
        __syncthreads();
        for (int j = wid; j < n; j += 4) {
            const int4 en = s_ent[j];
            const int c0 = en.y & 0xFFFF, r0 = (en.y >> 16) & 0xFFFF;
            const int nc = en.z & 255, nr = (en.z >> 8) & 255;
            const int lx0 = (en.z >> 16) & 255, ly0 = (en.z >> 24) & 255;
            const int jp = s_jp[j];
            const C *tp = taps + s_off[j] + (int64_t)r0 * jp + c0;
            const C y = s_y[j];
            const float inv_nc = 1.0f / (float)nc;
            const int ntap = nr * nc;
            for (int k0 = 0; k0 < ntap; k0 += 64 * kU) {
                C K[kU];
                int li[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int k = k0 + 64 * u + lane;
                    li[u] = -1;
                    if (k < ntap) {
                        // (k + 1/2) / nc is never within 1/(2 nc) of an integer: exact row
                        int row = (int)(((float)k + 0.5f) * inv_nc);
                        int col = k - row * nc;
                        K[u] = tp[row * jp + col];
                        li[u] = (ly0 + row) * kTile + lx0 + col;
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (li[u] >= 0) {
                        atomicAdd(&tre[li[u]], K[u].x * y.x + K[u].y * y.y);
                        atomicAdd(&tim[li[u]], K[u].x * y.y - K[u].y * y.x);
                    }
                }
            }
        }
    }
    __syncthreads();
    const uint32_t key = t.item_key[item];
    C *dst;
    int64_t ld;
    if (t.item_sole[item]) {
        // the tile's only item: store straight into the grid
        const int tmask = (1 << t.tile_bits) - 1;
        const int tx = key & tmask, ty = (key >> t.tile_bits) & tmask;
        const int k = key >> (2 * t.tile_bits);
        dst = grids + (int64_t)k * t.G * t.G + (int64_t)ty * kTile * t.G + (int64_t)tx * kTile;
        ld = t.G;
    } else {
        // a shared tile: store this item's partial tile; k_reduce_tiles sums them
        dst = (C *)t.partial + (int64_t)t.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
        C v;
        v.x = tre[i];
        v.y = tim[i];
        dst[(int64_t)(i / kTile) * ld + (i % kTile)] = v;
    }
}

// Sum the partial tiles of each tile shared by several items, in item order
// (deterministic), and store the result in the grid.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_reduce_tiles(const int32_t *__restrict__ mt_first,
                                                      typename Types<kFP64>::C *grids, TileArgs t) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const int a = mt_first[blockIdx.x];
    const uint32_t key = t.item_key[a];
    int b = a + 1;
    while (b < t.n_items && t.item_key[b] == key) ++b;
    const int slot0 = t.item_slot[a];
    const int tmask = (1 << t.tile_bits) - 1;
    const int tx = key & tmask, ty = (key >> t.tile_bits) & tmask;
    const int k = key >> (2 * t.tile_bits);
    C *dst = grids + (int64_t)k * t.G * t.G + (int64_t)ty * kTile * t.G + (int64_t)tx * kTile;
    const C *src = (const C *)t.partial + (int64_t)slot0 * kTile * kTile;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
        R vr = 0, vi = 0;
        for (int j = 0; j < b - a; ++j) {
            C v = src[(int64_t)j * kTile * kTile + i];
            vr += v.x;
            vi += v.y;
        }
        C o;
        o.x = vr;
        o.y = vi;
        dst[(int64_t)(i / kTile) * t.G + (i % kTile)] = o;
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
    unsigned nb = 8 * ((blocks(a.m * 64, 256) + 7) / 8);
    hipLaunchKernelGGL(k_degrid<kFP64>, dim3(nb), dim3(256), 0, s, (const C *)c->taps,
                       (const C *)c->grids, (C *)vis, a);
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
    const Plan &pl = c->plan;
    TileArgs ta{pl.ent,      pl.ent_sorted, pl.item_start, pl.item_key, pl.item_sole,
                pl.item_slot, c->scratch_part, pl.jp, pl.tap_off, pl.n_items, pl.tile_bits, g.G};
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_prep_vis<kFP64>, dim3(blocks(a.m, 256)), dim3(256), 0, s, (const C *)vis,
                       (C *)c->scratch_yw, a);
    if (pl.n_items > 0) {
        unsigned nb = (unsigned)(8 * ((pl.n_items + 7) / 8));
        hipLaunchKernelGGL(k_grid_tiles<kFP64>, dim3(nb), dim3(256), 0, s, (const C *)c->taps,
                           (const C *)c->scratch_yw, (C *)c->grids, ta);
    }
    if (pl.n_mtiles > 0) {
        hipLaunchKernelGGL(k_reduce_tiles<kFP64>, dim3(pl.n_mtiles), dim3(256), 0, s, pl.mt_first,
                           (C *)c->grids, ta);
    }
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
