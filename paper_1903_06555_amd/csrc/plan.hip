// Per-visibility planning on the GPU: conjugate-symmetry folding (Eq. (8)),
// k-means w-stacking (Algorithm 1), the support rule, the sort by
// (stack, grid tile) and the kernel-tap offsets.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <limits>

#include "wsp_internal.h"

namespace wsp {

namespace {

#define WSP_TRY(expr)                         \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

// ---------------------------------------------------------------- folding --
__global__ void k_fold(const double *__restrict__ uvw, const double *__restrict__ wts,
                       int64_t m, int fold, double *u, double *v, double *w, double *wt,
                       uint8_t *flag, int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double uu = uvw[3 * i], vv = uvw[3 * i + 1], ww = uvw[3 * i + 2];
    double wi = wts ? wts[i] : 1.0;
    if (!isfinite(uu) || !isfinite(vv) || !isfinite(ww) || !isfinite(wi)) atomicOr(bad, 1);
    // Eq. (8): y(u, v, w) = conj y(-u, -v, -w); strictly negative w is folded.
    bool f = fold && ww < 0.0;
    if (f) {
        uu = -uu;
        vv = -vv;
        ww = -ww;
    }
    u[i] = uu;
    v[i] = vv;
    w[i] = ww;
    wt[i] = wi;
    flag[i] = f ? 1 : 0;
}

// ----------------------------------------------------------- w min / max --
constexpr int kRedBlock = 256;

__global__ void k_minmax(const double *__restrict__ w, int64_t m, double *pmin, double *pmax) {
    __shared__ double smin[kRedBlock], smax[kRedBlock];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        double x = w[i];
        lo = fmin(lo, x);
        hi = fmax(hi, x);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmin[blockIdx.x] = smin[0];
        pmax[blockIdx.x] = smax[0];
    }
}

// ------------------------------------------------------------- k-means ----
// One Lloyd pass of Algorithm 1: each visibility takes the nearest centre
// (strict '<' in stack order, so ties keep the lowest stack), then every
// block writes its per-stack sum and count.  Sums are reduced in a fixed tree
// order inside a block and in block order afterwards, so results are
// reproducible run to run.
constexpr int kKmItems = 16;

__global__ void k_kmeans_assign(const double *__restrict__ w, int64_t m,
                                const double *__restrict__ centres, int K, int32_t *label,
                                double *psum, unsigned long long *pcnt) {
    __shared__ double rs[kRedBlock];
    __shared__ unsigned long long rc[kRedBlock];
    const int64_t base = (int64_t)blockIdx.x * kRedBlock * kKmItems;
    double wv[kKmItems];
    int lab[kKmItems];
#pragma unroll
    for (int it = 0; it < kKmItems; ++it) {
        int64_t idx = base + (int64_t)it * kRedBlock + threadIdx.x;
        lab[it] = -1;
        wv[it] = 0.0;
        if (idx < m) {
            double x = w[idx];
            double best = INFINITY;
            int l = 0;
            for (int q = 0; q < K; ++q) {
                double d = (centres[q] - x) * (centres[q] - x);
                if (d < best) {
                    best = d;
                    l = q;
                }
            }
            label[idx] = l;
            lab[it] = l;
            wv[it] = x;
        }
    }
    for (int q = 0; q < K; ++q) {
        double s = 0.0;
        unsigned long long cnt = 0;
#pragma unroll
        for (int it = 0; it < kKmItems; ++it) {
            if (lab[it] == q) {
                s += wv[it];
                ++cnt;
            }
        }
        rs[threadIdx.x] = s;
        rc[threadIdx.x] = cnt;
        __syncthreads();
        for (int st = kRedBlock / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) {
                rs[threadIdx.x] += rs[threadIdx.x + st];
                rc[threadIdx.x] += rc[threadIdx.x + st];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            psum[(int64_t)blockIdx.x * K + q] = rs[0];
            pcnt[(int64_t)blockIdx.x * K + q] = rc[0];
        }
        __syncthreads();
    }
}

// New centres (Algorithm 1): mean of each stack, 0 for an empty stack.
__global__ void k_kmeans_reduce(const double *__restrict__ psum,
                                const unsigned long long *__restrict__ pcnt, int nblk, int K,
                                double *centres) {
    int q = threadIdx.x;
    if (q >= K) return;
    double s = 0.0;
    unsigned long long c = 0;
    for (int b = 0; b < nblk; ++b) {
        s += psum[(int64_t)b * K + q];
        c += pcnt[(int64_t)b * K + q];
    }
    centres[q] = c > 0 ? s / (double)c : 0.0;
}

// ------------------------------------------------------- support + keys ---
struct SupportOut {
    double *ux, *vx, *weff;
    int32_t *jp, *u0w, *v0w;
    uint32_t *key;
};

__global__ void k_support(const double *__restrict__ u, const double *__restrict__ v,
                          const double *__restrict__ w, const int32_t *__restrict__ label,
                          const double *__restrict__ centres, int64_t m, Geom g, int max_support,
                          int tile_bits, SupportOut out, int *err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int lab = label[i];
    double weff = w[i] - centres[lab];
    // J_p = J + 2 ceil(|w - wbar| s f): FP64 product, rounded once.
    double half_extra = ceil(fabs(weff) * g.slope);
    if (!(half_extra <= (double)max_support)) {
        atomicOr(err, 1);
        half_extra = 0.0;
    }
    int jp = g.J + 2 * (int)half_extra;
    if (jp > max_support) {
        atomicOr(err, 1);
        jp = g.J;
    }
    double up = u[i] * g.inv_du;
    double vp = v[i] * g.inv_du;
    if (!(fabs(up) < 1.0e9) || !(fabs(vp) < 1.0e9)) {
        atomicOr(err, 2);
        up = 0.0;
        vp = 0.0;
    }
    int64_t u0 = (int64_t)floor(up) - jp / 2 + 1;
    int64_t v0 = (int64_t)floor(vp) - jp / 2 + 1;
    int64_t uw = u0 % g.G;
    if (uw < 0) uw += g.G;
    int64_t vw = v0 % g.G;
    if (vw < 0) vw += g.G;
    out.ux[i] = up - (double)u0;
    out.vx[i] = vp - (double)v0;
    out.weff[i] = weff;
    out.jp[i] = jp;
    out.u0w[i] = (int32_t)uw;
    out.v0w[i] = (int32_t)vw;
    uint32_t tx = (uint32_t)(uw / kTile), ty = (uint32_t)(vw / kTile);
    out.key[i] = ((uint32_t)lab << (2 * tile_bits)) | (ty << tile_bits) | tx;
}

template <typename T>
__global__ void k_gather(const int32_t *__restrict__ perm, const T *__restrict__ src, T *dst,
                         int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) dst[i] = src[perm[i]];
}

__global__ void k_iota(int32_t *x, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) x[i] = (int32_t)i;
}

__global__ void k_tap_counts(const int32_t *__restrict__ jp, int64_t m, int64_t *cnt,
                             uint32_t *cost_key) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > m) return;
    if (i == m) {
        cnt[i] = 0;
        return;
    }
    int64_t j = jp[i];
    cnt[i] = j * j;
    // build cost ~ taps x panels, panels ~ support; larger cost sorts first
    uint64_t cost = (uint64_t)(j * j) * (uint64_t)(j + 16);
    if (cost > 0xFFFFFFFFull) cost = 0xFFFFFFFFull;
    cost_key[i] = 0xFFFFFFFFu - (uint32_t)cost;
}

__global__ void k_max_jp(const int32_t *__restrict__ jp, int64_t m, int *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) atomicMax(out, jp[i]);
}

inline unsigned grid1d(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
}

}  // namespace

hipError_t launch_fold(const double *uvw, const double *wts, int64_t m, int fold, Plan &pl,
                       int *d_bad, hipStream_t s) {
    hipLaunchKernelGGL(k_fold, dim3(grid1d(m, 256)), dim3(256), 0, s, uvw, wts, m, fold, pl.u,
                       pl.v, pl.w, pl.wt_in, pl.flag, d_bad);
    return hipGetLastError();
}

hipError_t minmax_w(const Plan &pl, double *wmin, double *wmax, hipStream_t s) {
    const int nblk = 512;
    double *d = nullptr;
    WSP_TRY(hipMalloc(&d, sizeof(double) * 2 * nblk));
    hipLaunchKernelGGL(k_minmax, dim3(nblk), dim3(kRedBlock), 0, s, pl.w, pl.m, d, d + nblk);
    std::vector<double> h(2 * nblk);
    hipError_t e = hipMemcpyAsync(h.data(), d, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(d);
    if (e != hipSuccess) return e;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        lo = std::fmin(lo, h[b]);
        hi = std::fmax(hi, h[nblk + b]);
    }
    *wmin = lo;
    *wmax = hi;
    return hipSuccess;
}

hipError_t kmeans_iteration(const Plan &pl, const double *d_centres, int K, double *h_new,
                            hipStream_t s) {
    const int64_t per = (int64_t)kRedBlock * kKmItems;
    const int nblk = (int)((pl.m + per - 1) / per);
    double *psum = nullptr, *dnew = nullptr;
    unsigned long long *pcnt = nullptr;
    WSP_TRY(hipMalloc(&psum, sizeof(double) * (size_t)nblk * K));
    WSP_TRY(hipMalloc(&pcnt, sizeof(unsigned long long) * (size_t)nblk * K));
    WSP_TRY(hipMalloc(&dnew, sizeof(double) * K));
    hipLaunchKernelGGL(k_kmeans_assign, dim3(nblk), dim3(kRedBlock), 0, s, pl.w, pl.m, d_centres,
                       K, pl.label, psum, pcnt);
    hipLaunchKernelGGL(k_kmeans_reduce, dim3(1), dim3(64 * ((K + 63) / 64)), 0, s, psum, pcnt,
                       nblk, K, dnew);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h_new, dnew, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(psum);
    hipFree(pcnt);
    hipFree(dnew);
    return e;
}

static void free_sorted(Plan &pl) {
    hipFree(pl.perm);
    hipFree(pl.ux);
    hipFree(pl.vx);
    hipFree(pl.weff);
    hipFree(pl.wt);
    hipFree(pl.jp);
    hipFree(pl.u0w);
    hipFree(pl.v0w);
    hipFree(pl.stack);
    hipFree(pl.sflag);
    hipFree(pl.tap_off);
    hipFree(pl.border);
    hipFree(pl.stats);
    pl.stats = nullptr;
    pl.perm = nullptr;
    pl.ux = pl.vx = pl.weff = pl.wt = nullptr;
    pl.jp = pl.u0w = pl.v0w = pl.stack = pl.border = nullptr;
    pl.sflag = nullptr;
    pl.tap_off = nullptr;
}

hipError_t make_plan(wsp_ctx *c, const double *d_centres, hipStream_t s, int *support_err) {
    Plan &pl = c->plan;
    const Geom &g = c->g;
    const int64_t m = pl.m;
    *support_err = 0;
    free_sorted(pl);

    int tiles = g.G / kTile;
    int tile_bits = 0;
    while ((1 << tile_bits) < tiles) ++tile_bits;
    int stack_bits = 0;
    while ((1 << stack_bits) < g.n_stacks) ++stack_bits;
    const int key_bits = 2 * tile_bits + stack_bits;

    // caller-order temporaries
    SupportOut t{};
    uint32_t *key_sorted = nullptr, *cost = nullptr, *cost_sorted = nullptr;
    int32_t *iota = nullptr, *order_tmp = nullptr;
    int64_t *cnt = nullptr;
    int *d_err = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        hipFree(t.ux);
        hipFree(t.vx);
        hipFree(t.weff);
        hipFree(t.jp);
        hipFree(t.u0w);
        hipFree(t.v0w);
        hipFree(t.key);
        hipFree(key_sorted);
        hipFree(cost);
        hipFree(cost_sorted);
        hipFree(iota);
        hipFree(order_tmp);
        hipFree(cnt);
        hipFree(d_err);
        hipFree(tmp);
    };
#define WSP_STEP(expr)                 \
    do {                               \
        e = (expr);                    \
        if (e != hipSuccess) {         \
            cleanup();                 \
            return e;                  \
        }                              \
    } while (0)

    WSP_STEP(dalloc(&t.ux, m));
    WSP_STEP(dalloc(&t.vx, m));
    WSP_STEP(dalloc(&t.weff, m));
    WSP_STEP(dalloc(&t.jp, m));
    WSP_STEP(dalloc(&t.u0w, m));
    WSP_STEP(dalloc(&t.v0w, m));
    WSP_STEP(dalloc(&t.key, m));
    WSP_STEP(dalloc(&key_sorted, m));
    WSP_STEP(dalloc(&iota, m));
    WSP_STEP(dalloc(&d_err, 1));
    WSP_STEP(hipMemsetAsync(d_err, 0, sizeof(int), s));

    hipLaunchKernelGGL(k_support, dim3(grid1d(m, 256)), dim3(256), 0, s, pl.u, pl.v, pl.w,
                       pl.label, d_centres, m, g, c->p.max_support, tile_bits, t, d_err);
    WSP_STEP(hipGetLastError());
    int h_err = 0;
    WSP_STEP(hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    WSP_STEP(hipStreamSynchronize(s));
    if (h_err) {
        *support_err = h_err;
        cleanup();
        return hipSuccess;
    }

    // sort by (stack, tile of the first tap); values are caller indices
    WSP_STEP(dalloc(&pl.perm, m));
    hipLaunchKernelGGL(k_iota, dim3(grid1d(m, 256)), dim3(256), 0, s, iota, m);
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, t.key, key_sorted, iota,
                                                pl.perm, (int)m, 0, key_bits > 0 ? key_bits : 1, s));
    WSP_STEP(hipMalloc(&tmp, tmp_bytes));
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, t.key, key_sorted, iota, pl.perm,
                                                (int)m, 0, key_bits > 0 ? key_bits : 1, s));
    hipFree(tmp);
    tmp = nullptr;

    WSP_STEP(dalloc(&pl.ux, m));
    WSP_STEP(dalloc(&pl.vx, m));
    WSP_STEP(dalloc(&pl.weff, m));
    WSP_STEP(dalloc(&pl.wt, m));
    WSP_STEP(dalloc(&pl.jp, m));
    WSP_STEP(dalloc(&pl.u0w, m));
    WSP_STEP(dalloc(&pl.v0w, m));
    WSP_STEP(dalloc(&pl.stack, m));
    WSP_STEP(dalloc(&pl.sflag, m));
    WSP_STEP(dalloc(&pl.tap_off, m + 1));
    WSP_STEP(dalloc(&pl.border, m));
    WSP_STEP(dalloc(&pl.stats, 2));
    dim3 gb(grid1d(m, 256)), bb(256);
    hipLaunchKernelGGL(k_gather<double>, gb, bb, 0, s, pl.perm, t.ux, pl.ux, m);
    hipLaunchKernelGGL(k_gather<double>, gb, bb, 0, s, pl.perm, t.vx, pl.vx, m);
    hipLaunchKernelGGL(k_gather<double>, gb, bb, 0, s, pl.perm, t.weff, pl.weff, m);
    hipLaunchKernelGGL(k_gather<double>, gb, bb, 0, s, pl.perm, pl.wt_in, pl.wt, m);
    hipLaunchKernelGGL(k_gather<int32_t>, gb, bb, 0, s, pl.perm, t.jp, pl.jp, m);
    hipLaunchKernelGGL(k_gather<int32_t>, gb, bb, 0, s, pl.perm, t.u0w, pl.u0w, m);
    hipLaunchKernelGGL(k_gather<int32_t>, gb, bb, 0, s, pl.perm, t.v0w, pl.v0w, m);
    hipLaunchKernelGGL(k_gather<int32_t>, gb, bb, 0, s, pl.perm, pl.label, pl.stack, m);
    hipLaunchKernelGGL(k_gather<uint8_t>, gb, bb, 0, s, pl.perm, pl.flag, pl.sflag, m);
    WSP_STEP(hipGetLastError());

    // tap offsets (exclusive prefix of J_p^2) and the build order
    WSP_STEP(dalloc(&cnt, m + 1));
    WSP_STEP(dalloc(&cost, m));
    WSP_STEP(dalloc(&cost_sorted, m));
    hipLaunchKernelGGL(k_tap_counts, dim3(grid1d(m + 1, 256)), dim3(256), 0, s, pl.jp, m, cnt,
                       cost);
    WSP_STEP(hipGetLastError());
    tmp_bytes = 0;
    WSP_STEP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, pl.tap_off, (int)(m + 1), s));
    WSP_STEP(hipMalloc(&tmp, tmp_bytes));
    WSP_STEP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, pl.tap_off, (int)(m + 1), s));
    hipFree(tmp);
    tmp = nullptr;
    hipLaunchKernelGGL(k_iota, dim3(grid1d(m, 256)), dim3(256), 0, s, iota, m);
    tmp_bytes = 0;
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, cost, cost_sorted, iota,
                                                pl.border, (int)m, 0, 32, s));
    WSP_STEP(hipMalloc(&tmp, tmp_bytes));
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, cost, cost_sorted, iota,
                                                pl.border, (int)m, 0, 32, s));
    int64_t total = 0;
    WSP_STEP(hipMemcpyAsync(&total, pl.tap_off + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    WSP_STEP(hipMemsetAsync(d_err, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_max_jp, gb, bb, 0, s, pl.jp, m, d_err);
    int mx = 0;
    WSP_STEP(hipMemcpyAsync(&mx, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
    WSP_STEP(hipStreamSynchronize(s));
    pl.total_taps = total;
    pl.max_jp = mx;
    cleanup();
    return hipSuccess;
#undef WSP_STEP
}

}  // namespace wsp
