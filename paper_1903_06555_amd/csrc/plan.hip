// Per-visibility planning on the GPU: conjugate-symmetry folding (Eq. (8)),
// k-means w-stacking (Algorithm 1), the support rule, the sort by
// (stack, grid tile) and the kernel-tap offsets.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstring>
#include <limits>

#include "wsp_internal.h"
#include "wsp_plane.h"

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
    // one block per stack: strided partial sums, then a fixed-order tree
    // (deterministic for a given nblk)
    __shared__ double rs[kRedBlock];
    __shared__ unsigned long long rc[kRedBlock];
    const int q = blockIdx.x;
    double sm = 0.0;
    unsigned long long c = 0;
    for (int b = threadIdx.x; b < nblk; b += kRedBlock) {
        sm += psum[(int64_t)b * K + q];
        c += pcnt[(int64_t)b * K + q];
    }
    rs[threadIdx.x] = sm;
    rc[threadIdx.x] = c;
    __syncthreads();
    for (int st = kRedBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            rs[threadIdx.x] += rs[threadIdx.x + st];
            rc[threadIdx.x] += rc[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) centres[q] = rc[0] > 0 ? rs[0] / (double)rc[0] : 0.0;
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
    int jp = g.J + 2 * (int)half_extra + 2 * g.dde_h;  // + J_D - 1 with a DDE convolution
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

// inv[perm[i]] = i (caller index -> sorted index)
__global__ void k_invert(const int32_t *__restrict__ perm, int32_t *inv, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) inv[perm[i]] = (int32_t)i;
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
    return dmalloc((void **)p, sizeof(T) * (count ? count : 1));
}

// ------------------------------------------------ tile work lists ---------
// A visibility's J_p x J_p footprint, starting at the wrapped first tap
// (u0w, v0w), covers virtual tiles u0w / T .. (u0w + J_p - 1) / T (and the
// same in v); virtual tile t lands on physical tile t mod (G / T), which
// realises the circular convolution.  Each (visibility, tile) overlap is one
// entry holding the overlapping sub-block of the visibility's taps.
__global__ void k_entry_count(const int32_t *__restrict__ jp, const int32_t *__restrict__ u0w,
                              const int32_t *__restrict__ v0w, int64_t m, int64_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > m) return;
    if (i == m) {
        cnt[i] = 0;
        return;
    }
    int j = jp[i], u = u0w[i], v = v0w[i];
    int64_t ntx = (u + j - 1) / kTile - u / kTile + 1;
    int64_t nty = (v + j - 1) / kTile - v / kTile + 1;
    cnt[i] = ntx * nty;
}

__global__ void k_entry_fill(const int32_t *__restrict__ jp, const int32_t *__restrict__ u0w,
                             const int32_t *__restrict__ v0w, const int32_t *__restrict__ stack,
                             const int64_t *__restrict__ eoff, int64_t m, int n_tiles,
                             int tile_bits, int4 *ent, uint32_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int j = jp[i], u = u0w[i], v = v0w[i];
    const int tx0 = u / kTile, ty0 = v / kTile;
    const int ntx = (u + j - 1) / kTile - tx0 + 1;
    const int nty = (v + j - 1) / kTile - ty0 + 1;
    const uint32_t sk = (uint32_t)stack[i] << (2 * tile_bits);
    int64_t e = eoff[i];
    for (int iy = 0; iy < nty; ++iy) {
        int tvy = ty0 + iy;
        int r0 = tvy * kTile - v;
        r0 = r0 < 0 ? 0 : r0;
        int r1 = (tvy + 1) * kTile - v;
        r1 = r1 > j ? j : r1;
        int ly0 = v + r0 - tvy * kTile;
        uint32_t typ = (uint32_t)(tvy % n_tiles);
        for (int ix = 0; ix < ntx; ++ix) {
            int tvx = tx0 + ix;
            int c0 = tvx * kTile - u;
            c0 = c0 < 0 ? 0 : c0;
            int c1 = (tvx + 1) * kTile - u;
            c1 = c1 > j ? j : c1;
            int lx0 = u + c0 - tvx * kTile;
            uint32_t txp = (uint32_t)(tvx % n_tiles);
            uint32_t key = sk | (typ << tile_bits) | txp;
            ent[e] = make_int4((int)i, c0 | (r0 << 16),
                               (c1 - c0) | ((r1 - r0) << 8) | (lx0 << 16) | (ly0 << 24), (int)key);
            keys[e] = key;
            ++e;
        }
    }
}

// Per-entry records in work-list order, so that the tile kernels read their
// entries' metadata sequentially rather than through three gathers.
__global__ void k_entry_records(const int32_t *__restrict__ idx_sorted, const int4 *__restrict__ ent,
                                const int64_t *__restrict__ tap_off, const int32_t *__restrict__ jp,
                                int64_t E, int4 *wrec) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= E) return;
    const int4 en = ent[idx_sorted[s]];
    const int c0 = en.y & 0xFFFF, r0 = (en.y >> 16) & 0xFFFF, nr = (en.z >> 8) & 255;
    const int64_t first = tap_off[en.x] + blocked_entry_offset(r0, nr, c0, jp[en.x]);
    wrec[s] = make_int4((int)(uint32_t)first, (int)(first >> 32), en.z, en.x);
}

// w-plane kernels: sort key band | (stack, tile) key | pair row, with the pair
// row j = floor(|w_eff| / dw) of the entry's visibility and band =
// j / band_rows (8, 32 and 24 bits).
__global__ void k_entry_wkey(const uint32_t *__restrict__ keys, const int4 *__restrict__ ent,
                             const double *__restrict__ weff, double inv_dw, int band_rows, int64_t E,
                             uint64_t *k64) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double a = fmin(floor(fabs(weff[ent[e].x]) * inv_dw), 16777215.0);
    const uint64_t j = (uint64_t)a;
    uint64_t band = j / (uint64_t)band_rows;
    band = band > 255 ? 255 : band;
    k64[e] = (band << 56) | ((uint64_t)keys[e] << 24) | j;
}

__global__ void k_key_mid32(const uint64_t *__restrict__ k64, int64_t E, uint32_t *keys) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) keys[e] = (uint32_t)(k64[e] >> 24);
}

// Items grouped by tile (positions i of the stable key sort): sole flags,
// partial-slot demand and the first position of each split tile.
__global__ void k_group_flags(const uint32_t *__restrict__ ks, const int32_t *__restrict__ itile, int n,
                              uint8_t *sole, int *shared_pos, uint8_t *tile_head) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool first = i == 0 || ks[i] != ks[i - 1];
    const bool last = i == n - 1 || ks[i] != ks[i + 1];
    const bool multi = !(first && last);
    sole[itile[i]] = multi ? 0 : 1;
    shared_pos[i] = multi ? 1 : 0;
    tile_head[i] = (multi && first) ? 1 : 0;
}

__global__ void k_scatter_slot(const int32_t *__restrict__ itile, const int *__restrict__ pos, int n,
                               int32_t *slot) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) slot[itile[i]] = pos[i];
}

__global__ void k_entry_work(const uint32_t *__restrict__ keys_sorted,
                             const int32_t *__restrict__ idx_sorted, const int4 *__restrict__ ent,
                             int64_t E, int64_t *work, uint8_t *head) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= E) return;
    int z = ent[idx_sorted[s]].z;
    work[s] = (int64_t)(z & 255) * ((z >> 8) & 255);
    head[s] = (s == 0 || keys_sorted[s] != keys_sorted[s - 1]) ? 1 : 0;
}

__global__ void k_seg_base_cand(const int64_t *__restrict__ incl, const int64_t *__restrict__ work,
                                const uint8_t *__restrict__ head, int64_t E, int64_t *cand) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < E) cand[s] = head[s] ? incl[s] - work[s] : 0;
}

// An item starts where a tile starts or where the tap count since the tile
// start crosses a multiple of kItemTaps.
__global__ void k_item_head(const int64_t *__restrict__ incl, const int64_t *__restrict__ work,
                            const int64_t *__restrict__ segbase, const uint8_t *__restrict__ head,
                            int64_t E, int64_t item_taps, uint8_t *ihead) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= E) return;
    if (head[s]) {
        ihead[s] = 1;
        return;
    }
    int64_t c = (incl[s] - work[s] - segbase[s]) / item_taps;
    int64_t cp = (incl[s - 1] - work[s - 1] - segbase[s - 1]) / item_taps;
    ihead[s] = c != cp ? 1 : 0;
}

__global__ void k_item_info(const int32_t *__restrict__ item_start, int n_items, int64_t E,
                            const uint32_t *__restrict__ keys_sorted, uint32_t *item_key,
                            int32_t *item_start_out_last) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    item_key[i] = keys_sorted[item_start[i]];
    if (i == n_items - 1) *item_start_out_last = (int32_t)E;
}

// ------------------------------------------- band-major tap layout -------
// Bands [b0, b0 + nb) of br tile rows that an entry covers.
__device__ __forceinline__ void entry_bands(int z, int br, int *b0, int *nb) {
    const int nr = (z >> 8) & 255, ly0 = (z >> 24) & 255;
    *b0 = ly0 / br;
    *nb = (ly0 + nr - 1) / br - *b0 + 1;
}

__global__ void k_run_counts(const int4 *__restrict__ ent, int64_t E, int br, int32_t *cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > E) return;
    if (e == E) {
        cnt[e] = 0;
        return;
    }
    int b0, nb;
    entry_bands(ent[e].z, br, &b0, &nb);
    cnt[e] = nb;
}

__global__ void k_pos_of(const int32_t *__restrict__ ent_sorted, int64_t E, int32_t *pos_of) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < E) pos_of[ent_sorted[s]] = (int32_t)s;
}

// marks[item_start[i]] = 1 for i >= 1 (an inclusive scan then gives each
// work position its item)
__global__ void k_item_marks(const int32_t *__restrict__ item_start, int n_items, int32_t *marks) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 1 && i < n_items) marks[item_start[i]] = 1;
}

// Runs in generation order: sort key (item, band, longest first, then the
// run's shape: width and first cell), tap count and entry.  Runs of one
// shape (same width, rows and first cell, so the same cells) become
// neighbours, a "class".  Equal keys keep generation order (the radix sort
// is stable).
__global__ void k_run_keys(const int4 *__restrict__ ent, const int32_t *__restrict__ run_first,
                           const int32_t *__restrict__ pos_of, const int32_t *__restrict__ item_of_pos,
                           int64_t E, int br, uint64_t *key, int32_t *gidx, int32_t *rlen, int32_t *rent) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int z = ent[e].z;
    const int nc = z & 255, nr = (z >> 8) & 255, ly0 = (z >> 24) & 255;
    int b0, nb;
    entry_bands(z, br, &b0, &nb);
    const int32_t s = pos_of[e];
    const uint64_t it = (uint64_t)item_of_pos[s];
    for (int k = 0; k < nb; ++k) {
        const int b = b0 + k;
        const int g = run_first[e] + k;
        const int lo = ly0 > b * br ? ly0 : b * br;
        const int hi = (ly0 + nr < (b + 1) * br) ? ly0 + nr : (b + 1) * br;
        const int len = (hi - lo) * nc;  // <= 16 * 64
        const int cell0 = (lo - b * br) * kTile + ((z >> 16) & 255);
        key[g] = (it << 32) | ((uint64_t)b << 28) | ((uint64_t)(2047 - len) << 17) | ((uint64_t)nc << 10) |
                 (uint64_t)cell0;
        gidx[g] = g;
        rlen[g] = len;
        rent[g] = (int32_t)e;
    }
}

__device__ __forceinline__ int64_t run_unit(uint64_t key, int bands) {
    return (int64_t)(key >> 32) * bands + (int64_t)((key >> 28) & 15);
}

__global__ void k_run_lengths(const int32_t *__restrict__ lay2gen, const int32_t *__restrict__ rlen,
                              int64_t R, int64_t *len_lay) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L > R) return;
    len_lay[L] = L == R ? 0 : rlen[lay2gen[L]];
}

__global__ void k_run_taps(const int32_t *__restrict__ lay2gen, const int64_t *__restrict__ start_lay,
                           int64_t R, int64_t *run_tap) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L < R) run_tap[lay2gen[L]] = start_lay[L];
}

// Layout position of each generation-order run.
__global__ void k_run_slots(const int32_t *__restrict__ lay2gen, int64_t R, int32_t *run_lay) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L < R) run_lay[lay2gen[L]] = (int32_t)L;
}

// First run of each unit (units without runs take the next unit's first run).
__global__ void k_unit_heads(const uint64_t *__restrict__ keys, int64_t R, int64_t U, int bands,
                             int32_t *unit_run0) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= R) return;
    const int64_t u = run_unit(keys[L], bands);
    const int64_t up = L == 0 ? -1 : run_unit(keys[L - 1], bands);
    for (int64_t v = up + 1; v <= u; ++v) unit_run0[v] = (int32_t)L;
    if (L == R - 1)
        for (int64_t v = u + 1; v <= U; ++v) unit_run0[v] = (int32_t)R;
}

__global__ void k_unit_taps(const int32_t *__restrict__ unit_run0, const int64_t *__restrict__ start_lay,
                            int64_t U, int64_t *unit_tap0) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u <= U) unit_tap0[u] = start_lay[unit_run0[u]];
}

// Record of the run in layout position L, stored at slot[L] (or L).
__device__ __forceinline__ int4 run_record(uint64_t key, const int4 &en, int br, int rel, int gen) {
    const int b = (int)((key >> 28) & 15);
    const int z = en.z;
    const int nc = z & 255, nr = (z >> 8) & 255, lx0 = (z >> 16) & 255, ly0 = (z >> 24) & 255;
    const int lo = ly0 > b * br ? ly0 : b * br;
    const int hi = (ly0 + nr < (b + 1) * br) ? ly0 + nr : (b + 1) * br;
    const int cell0 = (lo - b * br) * kTile + lx0;
    return make_int4(rel, cell0 | (nc << 16) | ((hi - lo) << 24), en.x, gen);
}

__global__ void k_run_records(const uint64_t *__restrict__ keys, const int32_t *__restrict__ lay2gen,
                              const int64_t *__restrict__ start_lay, const int64_t *__restrict__ unit_tap0,
                              const int32_t *__restrict__ rent, const int4 *__restrict__ ent, int64_t R,
                              int br, int4 *runrec) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= R) return;
    const uint64_t key = keys[L];
    const int g = lay2gen[L];
    runrec[L] = run_record(key, ent[rent[g]], br, (int)(start_lay[L] - unit_tap0[run_unit(key, kTile / br)]), g);
}

// ---- run classes (contiguous-runs layout): neighbouring runs of one shape
__global__ void k_class_heads(const uint64_t *__restrict__ keys, int64_t R, int32_t *head) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L < R) head[L] = (L == 0 || keys[L] != keys[L - 1]) ? 1 : 0;
}

// Class of each head run (inclusive scan of the heads, minus one): its first
// run and that run's key.
__global__ void k_class_first(const int32_t *__restrict__ head, const int32_t *__restrict__ cls_incl,
                              const uint64_t *__restrict__ keys, int64_t R, int32_t *cls_run0, uint64_t *cls_key) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= R || !head[L]) return;
    const int c = cls_incl[L] - 1;
    cls_run0[c] = (int32_t)L;
    cls_key[c] = keys[L];
}

// clsrec[c] = {first tap relative to the unit, first run, runs, cell0 | nc << 16 | nrows << 24}.
__global__ void k_class_records(const int32_t *__restrict__ cls_run0, const uint64_t *__restrict__ cls_key,
                                const int4 *__restrict__ runrec, int64_t n_cls, int64_t R, int4 *clsrec) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cls) return;
    const int r0 = cls_run0[c];
    const int r1 = c + 1 < n_cls ? cls_run0[c + 1] : (int)R;
    const int4 rr = runrec[r0];
    clsrec[c] = make_int4(rr.x, r0, r1 - r0, rr.y);
}

// Sort keys for the band order of the class kernels: the band's taps (to be
// sorted in decreasing order) and its index.
__global__ void k_unit_sizes(const int64_t *__restrict__ unit_tap0, int64_t U, int64_t *sz, int32_t *idx) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= U) return;
    sz[u] = unit_tap0[u + 1] - unit_tap0[u];
    idx[u] = (int32_t)u;
}

// Taps in classes whose shape has more than 64 taps.
__global__ void k_long_taps(const int4 *__restrict__ clsrec, int64_t n_cls, unsigned long long *out) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (c < n_cls) {
        const int4 cr = clsrec[c];
        const int L = ((cr.w >> 16) & 255) * ((cr.w >> 24) & 255);
        if (L > 64) v = (unsigned long long)L * (unsigned long long)cr.z;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

// ---- interleaved variant: units padded to whole groups of 64 runs
__global__ void k_padded_counts(const int32_t *__restrict__ unit_run0, int64_t U, int64_t *cnt) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > U) return;
    cnt[u] = u == U ? 0 : ((unit_run0[u + 1] - unit_run0[u] + 63) & ~63);
}

// Slot of sorted run L, its length and record (.x set by k_group_bases);
// the unit of each group's first slot.
__global__ void k_pad_scatter(const uint64_t *__restrict__ keys, const int32_t *__restrict__ lay2gen,
                              const int32_t *__restrict__ unit_run0, const int64_t *__restrict__ pad0,
                              const int32_t *__restrict__ rlen, const int32_t *__restrict__ rent,
                              const int4 *__restrict__ ent, int64_t R, int br, int32_t *run_lay,
                              uint16_t *len16, int4 *runrec, int32_t *grp_unit) {
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= R) return;
    const uint64_t key = keys[L];
    const int64_t u = run_unit(key, kTile / br);
    const int64_t slot = pad0[u] + (L - unit_run0[u]);
    const int g = lay2gen[L];
    run_lay[g] = (int32_t)slot;
    len16[slot] = (uint16_t)rlen[g];
    runrec[slot] = run_record(key, ent[rent[g]], br, 0, g);
    if ((slot & 63) == 0) grp_unit[slot >> 6] = (int32_t)u;
}

// Per group: suffix sums of the lengths, the group's taps and its longest run
// (slot 0: lengths are sorted longest first).
__global__ void k_group_sums(const uint16_t *__restrict__ len16, int64_t n_groups, uint32_t *suf,
                             int64_t *grp_len, unsigned long long *steps) {
    int64_t G = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (G > n_groups) return;
    if (G == n_groups) {
        grp_len[G] = 0;
        return;
    }
    uint32_t acc = 0;
    for (int j = 63; j >= 0; --j) {
        acc += len16[G * 64 + j];
        suf[G * 64 + j] = acc;
    }
    grp_len[G] = acc;
    atomicAdd(steps, (unsigned long long)len16[G * 64]);
}

__global__ void k_unit_taps_padded(const int64_t *__restrict__ pad0, const int64_t *__restrict__ grp_tap,
                                   int64_t U, int64_t *unit_tap0, int32_t *unit_run0) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > U) return;
    unit_tap0[u] = grp_tap[pad0[u] >> 6];
    unit_run0[u] = (int32_t)pad0[u];  // units now start at their padded slots
}

// .x of every slot of group G: the group's first tap relative to its unit
// (slot 0 of a group always holds a run: a unit's runs fill its first slots).
__global__ void k_group_bases(const int64_t *__restrict__ grp_tap, const int64_t *__restrict__ unit_tap0,
                              const int32_t *__restrict__ grp_unit, int64_t n_groups, int4 *runrec) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_groups * 64) return;
    const int64_t G = t >> 6;
    runrec[t].x = (int)(grp_tap[G] - unit_tap0[grp_unit[G]]);
}

__global__ void k_fill_padding(int64_t n, int4 *runrec) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) runrec[t] = make_int4(0, 0, 0, -1);
}

// Touched cells: every row of an entry covers columns lx0 .. lx0 + nc - 1 of
// one tile row, a bit range of that tile row's 64-bit word.
__global__ void k_touched_rows(const int4 *__restrict__ ent, int64_t E, unsigned long long *words) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int4 en = ent[e];
    const int nc = en.z & 255, nr = (en.z >> 8) & 255, lx0 = (en.z >> 16) & 255, ly0 = (en.z >> 24) & 255;
    const unsigned long long bits = (nc >= 64 ? ~0ull : ((1ull << nc) - 1ull)) << lx0;
    unsigned long long *w = words + (int64_t)(uint32_t)en.w * kTile + ly0;
    for (int r = 0; r < nr; ++r) atomicOr(w + r, bits);
}

__global__ void k_popcount_sum(const unsigned long long *__restrict__ words, int64_t n,
                               unsigned long long *total) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += (unsigned long long)__popcll(words[i]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(total, c);
}

__global__ void k_find_index(const int32_t *__restrict__ perm, int64_t m, int32_t p, int64_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && perm[i] == p) *out = i;  // perm is a permutation: one writer
}

}  // namespace

hipError_t find_sorted_index(const wsp_ctx *c, int64_t p, int64_t *sidx) {
    int64_t *d = nullptr;
    *sidx = -1;
    hipError_t e = dmalloc(&d, sizeof(int64_t));
    if (e == hipSuccess) e = hipMemcpy(d, sidx, sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_find_index, dim3(grid1d(c->plan.m, 256)), dim3(256), 0, 0, c->plan.perm, c->plan.m,
                           (int32_t)p, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(sidx, d, sizeof(int64_t), hipMemcpyDeviceToHost);
    dfree(d);
    return e;
}

hipError_t count_touched_cells(const wsp_ctx *c, int64_t *cells) {
    const Plan &pl = c->plan;
    int stack_bits = 0;
    while ((1 << stack_bits) < c->g.n_stacks) ++stack_bits;
    const int64_t n_words = ((int64_t)1 << (2 * pl.tile_bits + stack_bits)) * kTile;
    unsigned long long *words = nullptr, *total = nullptr;
    hipError_t e = dmalloc(&words, sizeof(unsigned long long) * (size_t)n_words);
    if (e == hipSuccess) e = dmalloc(&total, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(words, 0, sizeof(unsigned long long) * (size_t)n_words);
    if (e == hipSuccess) e = hipMemset(total, 0, sizeof(unsigned long long));
    if (e == hipSuccess && pl.n_entries > 0) {
        hipLaunchKernelGGL(k_touched_rows, dim3(grid1d(pl.n_entries, 256)), dim3(256), 0, 0, pl.ent,
                           pl.n_entries, words);
        hipLaunchKernelGGL(k_popcount_sum, dim3(1024), dim3(256), 0, 0, words, n_words, total);
        e = hipGetLastError();
    }
    unsigned long long h = 0;
    if (e == hipSuccess) e = hipMemcpy(&h, total, sizeof(h), hipMemcpyDeviceToHost);
    dfree(words);
    dfree(total);
    *cells = (int64_t)h;
    return e;
}

hipError_t launch_fold(const double *uvw, const double *wts, int64_t m, int fold, Plan &pl,
                       int *d_bad, hipStream_t s) {
    hipLaunchKernelGGL(k_fold, dim3(grid1d(m, 256)), dim3(256), 0, s, uvw, wts, m, fold, pl.u,
                       pl.v, pl.w, pl.wt_in, pl.flag, d_bad);
    return hipGetLastError();
}

hipError_t minmax_w(const Plan &pl, double *wmin, double *wmax, hipStream_t s) {
    const int nblk = 512;
    double *d = nullptr;
    WSP_TRY(dmalloc(&d, sizeof(double) * 2 * nblk));
    hipLaunchKernelGGL(k_minmax, dim3(nblk), dim3(kRedBlock), 0, s, pl.w, pl.m, d, d + nblk);
    std::vector<double> h(2 * nblk);
    hipError_t e = hipMemcpyAsync(h.data(), d, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(d);
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
    WSP_TRY(dmalloc(&psum, sizeof(double) * (size_t)nblk * K));
    WSP_TRY(dmalloc(&pcnt, sizeof(unsigned long long) * (size_t)nblk * K));
    WSP_TRY(dmalloc(&dnew, sizeof(double) * K));
    hipLaunchKernelGGL(k_kmeans_assign, dim3(nblk), dim3(kRedBlock), 0, s, pl.w, pl.m, d_centres,
                       K, pl.label, psum, pcnt);
    hipLaunchKernelGGL(k_kmeans_reduce, dim3(K), dim3(kRedBlock), 0, s, psum, pcnt, nblk, K, dnew);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h_new, dnew, sizeof(double) * K, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(psum);
    dfree(pcnt);
    dfree(dnew);
    return e;
}

void free_sorted_plan(Plan &pl) {
    void *ptrs[] = {pl.perm,   pl.ux,      pl.vx,         pl.weff,     pl.wt,
                    pl.jp,     pl.u0w,     pl.v0w,        pl.stack,    pl.sflag,
                    pl.tap_off, pl.border, pl.stats,      pl.ent,      pl.ent_off,
                    pl.ent_sorted, pl.item_start, pl.item_key, pl.item_sole, pl.wrec, pl.iperm};
    for (void *q : ptrs) dfree(q);
    pl.perm = pl.iperm = nullptr;
    pl.ux = pl.vx = pl.weff = pl.wt = nullptr;
    pl.jp = pl.u0w = pl.v0w = pl.stack = pl.border = nullptr;
    pl.sflag = nullptr;
    pl.tap_off = nullptr;
    pl.stats = nullptr;
    pl.ent = nullptr;
    pl.ent_off = nullptr;
    pl.ent_sorted = pl.item_start = nullptr;
    pl.wrec = nullptr;
    pl.item_key = nullptr;
    pl.item_sole = nullptr;
    pl.n_entries = 0;
    pl.n_items = 0;
    dfree(pl.item_slot);
    dfree(pl.mt_first);
    dfree(pl.itile);
    pl.item_slot = pl.mt_first = pl.itile = nullptr;
    pl.n_multi = pl.n_mtiles = 0;
    dfree(pl.plane_off);
    dfree(pl.prec);
    dfree(pl.ptw);
    pl.plane_off = nullptr;
    pl.prec = nullptr;
    pl.ptw = nullptr;
    pl.n_pairs = 0;
    pl.table_len = 0;
    void *rptrs[] = {pl.run_first, pl.run_tap, pl.runrec,  pl.unit_run0, pl.unit_tap0,  pl.run_lay,
                     pl.len16,     pl.suf,     pl.grp_tap, pl.clsrec,    pl.unit_cls0, pl.unit_order};
    for (void *q : rptrs) dfree(q);
    pl.run_first = pl.unit_run0 = pl.run_lay = pl.unit_cls0 = pl.unit_order = nullptr;
    pl.clsrec = nullptr;
    pl.n_classes = 0;
    pl.long_taps = 0;
    pl.run_tap = pl.unit_tap0 = pl.grp_tap = nullptr;
    pl.runrec = nullptr;
    pl.len16 = nullptr;
    pl.suf = nullptr;
    pl.n_runs = pl.n_runs_padded = pl.group_steps = 0;
    pl.interleaved = false;
}

// ---- w-plane mode ---------------------------------------------------------------

// max |w_eff| as the bit pattern of a non-negative double (ordered like the value)
__global__ void k_absmax_weff(const double *__restrict__ weff, int64_t m, unsigned long long *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (i < m) v = (unsigned long long)__double_as_longlong(fabs(weff[i]));
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

// Per entry (work-list order): the pair row of its visibility's |w_eff|, the
// w weight, the conjugation flag and the visibility's offset from the
// entry's first tap.
__global__ void k_plane_records(const int32_t *__restrict__ idx_sorted, const int4 *__restrict__ ent,
                                const double *__restrict__ ux, const double *__restrict__ vx,
                                const double *__restrict__ weff, const int64_t *__restrict__ plane_off,
                                int n_pairs, double inv_dw, int64_t E, int4 *prec, float *ptw) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= E) return;
    const int4 en = ent[idx_sorted[s]];
    const int p = en.x;
    const int c0 = en.y & 0xFFFF, r0 = (en.y >> 16) & 0xFFFF;
    plane_record(weff[p], ux[p] - (double)c0, vx[p] - (double)r0, plane_off, n_pairs, inv_dw,
                 &prec[s], &ptw[s]);
}

// Lattice layout for the planned visibilities (host arithmetic in FP64).
// Pair row j serves |w_eff| in [j dw, (j + 1) dw): its supports are at most
// J_p((j + 1) dw), whose taps lie within J_p / sqrt(2) cells of the
// visibility.  Also chooses the bands of the work order (below), so that the
// lattice rows in use at a time stay in cache.
hipError_t plane_layout(wsp_ctx *c, hipStream_t s, bool *too_large) {
    Plan &pl = c->plan;
    const Geom &g = c->g;
    *too_large = false;
    unsigned long long *d_max = nullptr;
    hipError_t e = dalloc(&d_max, 1);
    if (e != hipSuccess) return e;
    unsigned long long h_max = 0;
    e = hipMemsetAsync(d_max, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_absmax_weff, dim3(grid1d(pl.m, 256)), dim3(256), 0, s, pl.weff, pl.m, d_max);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h_max, d_max, sizeof(h_max), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(d_max);
    if (e != hipSuccess) return e;
    double wmax;
    static_assert(sizeof(wmax) == sizeof(h_max), "bit pattern");
    memcpy(&wmax, &h_max, sizeof(wmax));
    const double npairs_d = floor(wmax * g.plane_inv_dw) + 1.0;
    if (!(npairs_d < 1.0e7)) {
        *too_large = true;
        return hipSuccess;
    }
    const int n_pairs = (int)npairs_d;
    std::vector<int64_t> off((size_t)n_pairs + 1);
    int64_t tot = 0;
    for (int j = 0; j < n_pairs; ++j) {
        off[j] = tot;
        const double w_hi = (double)(j + 1) * c->g.plane_dw * (1.0 + 1e-12) + 1e-12;
        double jp = (double)g.J + 2.0 * ceil(w_hi * g.slope);
        if (jp > (double)c->p.max_support) jp = (double)c->p.max_support;
        tot += (int64_t)floor(jp * 0.70710678118654757 * g.plane_inv_dq) + 3;
    }
    off[n_pairs] = tot;
    if (tot >= (int64_t)0x7FFFFFF0) {  // row offsets are stored as int32
        *too_large = true;
        return hipSuccess;
    }
    pl.n_pairs = n_pairs;
    pl.table_len = tot;
    // a lattice that fits the last-level cache needs no bands (they would only
    // add items and partial tiles); a larger one is cut into bands of about
    // one XCD's L2 (4 MiB), at most 255
    const int64_t bytes = tot * 16, band_bytes = (int64_t)4 << 20;
    int64_t nbands = bytes <= ((int64_t)64 << 20) ? 1 : (bytes + band_bytes - 1) / band_bytes;
    nbands = nbands > 255 ? 255 : nbands;
    pl.band_rows = (int)((n_pairs + nbands - 1) / nbands);
    e = dalloc(&pl.plane_off, (size_t)n_pairs + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl.plane_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // off[] is released on return
    return e;
}

// Per-entry plane records (work-list order), after the work lists.
hipError_t plane_setup(wsp_ctx *c, hipStream_t s) {
    Plan &pl = c->plan;
    const Geom &g = c->g;
    const int64_t E = pl.n_entries;
    hipError_t e = dalloc(&pl.prec, (size_t)(E > 0 ? E : 1));
    if (e == hipSuccess) e = dalloc(&pl.ptw, (size_t)(E > 0 ? E : 1));
    if (e == hipSuccess && E > 0) {
        hipLaunchKernelGGL(k_plane_records, dim3(grid1d(E, 256)), dim3(256), 0, s, pl.ent_sorted, pl.ent,
                           pl.ux, pl.vx, pl.weff, pl.plane_off, pl.n_pairs, g.plane_inv_dw, E, pl.prec,
                           pl.ptw);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Tile work lists of the sorted visibilities (see k_entry_fill).
static hipError_t make_entries(Plan &pl, const Geom &g, int tile_bits, hipStream_t s) {
    const int64_t m = pl.m;
    const int n_tiles = g.G / kTile;
    int64_t *cnt = nullptr, *work = nullptr, *incl = nullptr, *cand = nullptr, *segbase = nullptr;
    uint32_t *keys = nullptr, *keys_sorted = nullptr;
    int32_t *iota = nullptr, *d_nsel = nullptr;
    uint8_t *head = nullptr, *ihead = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        void *ptrs[] = {cnt, work, incl, cand, segbase, keys, keys_sorted, iota, d_nsel, head, ihead, tmp};
        for (void *q : ptrs) dfree(q);
    };
#define WSP_ESTEP(expr)        \
    do {                       \
        e = (expr);            \
        if (e != hipSuccess) { \
            cleanup();         \
            return e;          \
        }                      \
    } while (0)
    auto scratch = [&](size_t need) -> hipError_t {
        if (need <= tmp_bytes && tmp) return hipSuccess;
        dfree(tmp);
        tmp = nullptr;
        tmp_bytes = need;
        return dmalloc(&tmp, need ? need : 1);
    };
    size_t need = 0;

    WSP_ESTEP(dalloc(&cnt, m + 1));
    WSP_ESTEP(dalloc(&pl.ent_off, m + 1));
    hipLaunchKernelGGL(k_entry_count, dim3(grid1d(m + 1, 256)), dim3(256), 0, s, pl.jp, pl.u0w,
                       pl.v0w, m, cnt);
    WSP_ESTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, need, cnt, pl.ent_off, (int)(m + 1), s));
    WSP_ESTEP(scratch(need));
    WSP_ESTEP(hipcub::DeviceScan::ExclusiveSum(tmp, need, cnt, pl.ent_off, (int)(m + 1), s));
    int64_t E = 0;
    WSP_ESTEP(hipMemcpyAsync(&E, pl.ent_off + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    WSP_ESTEP(hipStreamSynchronize(s));
    if (E >= 0x7FFFFFF0LL) {
        cleanup();
        return hipErrorInvalidValue;
    }
    pl.n_entries = E;

    WSP_ESTEP(dalloc(&pl.ent, E));
    WSP_ESTEP(dalloc(&keys, E));
    WSP_ESTEP(dalloc(&keys_sorted, E));
    WSP_ESTEP(dalloc(&iota, E));
    WSP_ESTEP(dalloc(&pl.ent_sorted, E));
    hipLaunchKernelGGL(k_entry_fill, dim3(grid1d(m, 256)), dim3(256), 0, s, pl.jp, pl.u0w, pl.v0w,
                       pl.stack, pl.ent_off, m, n_tiles, tile_bits, pl.ent, keys);
    hipLaunchKernelGGL(k_iota, dim3(grid1d(E, 256)), dim3(256), 0, s, iota, E);
    WSP_ESTEP(hipGetLastError());
    int stack_bits = 0;
    while ((1 << stack_bits) < g.n_stacks) ++stack_bits;
    int key_bits = 2 * tile_bits + stack_bits;
    key_bits = key_bits > 0 ? key_bits : 1;
    if (g.planes) {
        // w-plane kernels: entries in bands of |w_eff| (each band's lattice rows
        // fit an XCD's L2; one band when the whole lattice fits the last-level
        // cache), within a band by tile, within a tile by lattice pair row, so
        // concurrent blocks and neighbouring wavefronts read the same lattice
        // rows.  A tile then has one item per band.
        uint64_t *k64 = nullptr, *k64s = nullptr;
        WSP_ESTEP(dalloc(&k64, E));
        hipError_t e2 = dalloc(&k64s, E);
        if (e2 == hipSuccess) {
            hipLaunchKernelGGL(k_entry_wkey, dim3(grid1d(E, 256)), dim3(256), 0, s, keys, pl.ent, pl.weff,
                               g.plane_inv_dw, pl.band_rows, E, k64);
            e2 = hipGetLastError();
        }
        size_t need64 = 0;
        if (e2 == hipSuccess)
            e2 = hipcub::DeviceRadixSort::SortPairs(nullptr, need64, k64, k64s, iota, pl.ent_sorted, (int)E,
                                                    0, 64, s);
        if (e2 == hipSuccess) e2 = scratch(need64);
        if (e2 == hipSuccess)
            e2 = hipcub::DeviceRadixSort::SortPairs(tmp, need64, k64, k64s, iota, pl.ent_sorted, (int)E, 0,
                                                    64, s);
        if (e2 == hipSuccess) {
            hipLaunchKernelGGL(k_key_mid32, dim3(grid1d(E, 256)), dim3(256), 0, s, k64s, E, keys_sorted);
            e2 = hipGetLastError();
        }
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);  // before k64 / k64s are released
        dfree(k64);
        dfree(k64s);
        WSP_ESTEP(e2);
    } else {
        need = 0;
        WSP_ESTEP(hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys_sorted, iota,
                                                     pl.ent_sorted, (int)E, 0, key_bits, s));
        WSP_ESTEP(scratch(need));
        WSP_ESTEP(hipcub::DeviceRadixSort::SortPairs(tmp, need, keys, keys_sorted, iota, pl.ent_sorted,
                                                     (int)E, 0, key_bits, s));
    }

    // work items: cut each tile's entries every g.item_taps taps
    WSP_ESTEP(dalloc(&work, E));
    WSP_ESTEP(dalloc(&incl, E));
    WSP_ESTEP(dalloc(&cand, E));
    WSP_ESTEP(dalloc(&segbase, E));
    WSP_ESTEP(dalloc(&head, E));
    WSP_ESTEP(dalloc(&ihead, E));
    hipLaunchKernelGGL(k_entry_work, dim3(grid1d(E, 256)), dim3(256), 0, s, keys_sorted,
                       pl.ent_sorted, pl.ent, E, work, head);
    if (g.planes) {  // entry records of the w-plane kernels
        WSP_ESTEP(dalloc(&pl.wrec, E));
        hipLaunchKernelGGL(k_entry_records, dim3(grid1d(E, 256)), dim3(256), 0, s, pl.ent_sorted, pl.ent,
                           pl.tap_off, pl.jp, E, pl.wrec);
    }
    need = 0;
    WSP_ESTEP(hipcub::DeviceScan::InclusiveSum(nullptr, need, work, incl, (int)E, s));
    WSP_ESTEP(scratch(need));
    WSP_ESTEP(hipcub::DeviceScan::InclusiveSum(tmp, need, work, incl, (int)E, s));
    hipLaunchKernelGGL(k_seg_base_cand, dim3(grid1d(E, 256)), dim3(256), 0, s, incl, work, head,
                       E, cand);
    need = 0;
    WSP_ESTEP(hipcub::DeviceScan::InclusiveScan(nullptr, need, cand, segbase, hipcub::Max(), (int)E, s));
    WSP_ESTEP(scratch(need));
    WSP_ESTEP(hipcub::DeviceScan::InclusiveScan(tmp, need, cand, segbase, hipcub::Max(), (int)E, s));
    hipLaunchKernelGGL(k_item_head, dim3(grid1d(E, 256)), dim3(256), 0, s, incl, work, segbase,
                       head, E, g.item_taps, ihead);
    WSP_ESTEP(hipGetLastError());
    // item starts = indices s with ihead[s] = 1 (at most E items)
    WSP_ESTEP(dalloc(&pl.item_start, E + 1));
    WSP_ESTEP(dalloc(&d_nsel, 1));
    hipcub::CountingInputIterator<int32_t> counting(0);
    need = 0;
    WSP_ESTEP(hipcub::DeviceSelect::Flagged(nullptr, need, counting, ihead, pl.item_start, d_nsel,
                                            (int)E, s));
    WSP_ESTEP(scratch(need));
    WSP_ESTEP(hipcub::DeviceSelect::Flagged(tmp, need, counting, ihead, pl.item_start, d_nsel,
                                            (int)E, s));
    int nsel = 0;
    WSP_ESTEP(hipMemcpyAsync(&nsel, d_nsel, sizeof(int), hipMemcpyDeviceToHost, s));
    WSP_ESTEP(hipStreamSynchronize(s));
    pl.n_items = nsel;
    WSP_ESTEP(dalloc(&pl.item_key, nsel));
    WSP_ESTEP(dalloc(&pl.item_sole, nsel));
    hipLaunchKernelGGL(k_item_info, dim3(grid1d(nsel, 256)), dim3(256), 0, s, pl.item_start, nsel,
                       E, keys_sorted, pl.item_key, pl.item_start + nsel);
    WSP_ESTEP(hipGetLastError());
    // items of tiles split over several items write partial tiles to slots;
    // a tile's items are grouped by a stable sort on the key (the identity
    // when the work order is by tile), slots follow that grouping, and the
    // split tiles' first positions index the reduction
    {
        int *shared_pos = nullptr, *slot_pos = nullptr;
        uint32_t *iks = nullptr;
        int32_t *iiota = nullptr;
        WSP_ESTEP(dalloc(&shared_pos, nsel + 1));
        WSP_ESTEP(dalloc(&slot_pos, nsel + 1));
        WSP_ESTEP(dalloc(&iks, nsel));
        WSP_ESTEP(dalloc(&iiota, nsel));
        WSP_ESTEP(dalloc(&pl.itile, nsel));
        WSP_ESTEP(dalloc(&pl.item_slot, nsel + 1));
        WSP_ESTEP(dalloc(&pl.mt_first, nsel + 1));
        uint8_t *tile_head = ihead;  // reuse (E >= nsel)
        hipLaunchKernelGGL(k_iota, dim3(grid1d(nsel, 256)), dim3(256), 0, s, iiota, (int64_t)nsel);
        e = hipGetLastError();
        if (e == hipSuccess) {
            need = 0;
            e = hipcub::DeviceRadixSort::SortPairs(nullptr, need, pl.item_key, iks, iiota, pl.itile, nsel, 0,
                                                   key_bits, s);
        }
        if (e == hipSuccess) e = scratch(need);
        if (e == hipSuccess)
            e = hipcub::DeviceRadixSort::SortPairs(tmp, need, pl.item_key, iks, iiota, pl.itile, nsel, 0,
                                                   key_bits, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_group_flags, dim3(grid1d(nsel, 256)), dim3(256), 0, s, iks, pl.itile, nsel,
                               pl.item_sole, shared_pos, tile_head);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemsetAsync(shared_pos + nsel, 0, sizeof(int), s);
        if (e == hipSuccess) {
            need = 0;
            e = hipcub::DeviceScan::ExclusiveSum(nullptr, need, shared_pos, slot_pos, nsel + 1, s);
        }
        if (e == hipSuccess) e = scratch(need);
        if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(tmp, need, shared_pos, slot_pos, nsel + 1, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_scatter_slot, dim3(grid1d(nsel, 256)), dim3(256), 0, s, pl.itile, slot_pos,
                               nsel, pl.item_slot);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            need = 0;
            e = hipcub::DeviceSelect::Flagged(nullptr, need, counting, tile_head, pl.mt_first, d_nsel,
                                              nsel, s);
        }
        if (e == hipSuccess) e = scratch(need);
        if (e == hipSuccess)
            e = hipcub::DeviceSelect::Flagged(tmp, need, counting, tile_head, pl.mt_first, d_nsel,
                                              nsel, s);
        int nmt = 0, nmulti = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&nmt, d_nsel, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nmulti, slot_pos + nsel, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pl.mt_first + nmt, &nsel, sizeof(int), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(shared_pos);
        dfree(slot_pos);
        dfree(iks);
        dfree(iiota);
        WSP_ESTEP(e);
        pl.n_mtiles = nmt;
        pl.n_multi = nmulti;
    }
    cleanup();
    return hipSuccess;
#undef WSP_ESTEP
}

// The interleaved tap layout (see Plan) from the runs in sorted order:
// units padded to whole groups, groups' tap offsets and suffix sums, records.
static hipError_t make_interleaved(Plan &pl, int64_t R, int64_t U, const uint64_t *key_sorted,
                                   const int32_t *lay2gen, const int32_t *rlen, const int32_t *rent,
                                   hipStream_t s) {
    int64_t *cnt = nullptr, *pad0 = nullptr, *grp_len = nullptr;
    int32_t *grp_unit = nullptr;
    unsigned long long *steps = nullptr;
    void *tmp = nullptr;
    size_t need = 0;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        void *ptrs[] = {cnt, pad0, grp_len, grp_unit, steps, tmp};
        for (void *q : ptrs) dfree(q);
    };
#define WSP_ISTEP(expr)        \
    do {                       \
        e = (expr);            \
        if (e != hipSuccess) { \
            cleanup();         \
            return e;          \
        }                      \
    } while (0)
    WSP_ISTEP(dalloc(&cnt, U + 1));
    WSP_ISTEP(dalloc(&pad0, U + 1));
    hipLaunchKernelGGL(k_padded_counts, dim3(grid1d(U + 1, 256)), dim3(256), 0, s, pl.unit_run0, U, cnt);
    WSP_ISTEP(hipGetLastError());
    WSP_ISTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, need, cnt, pad0, (int)(U + 1), s));
    WSP_ISTEP(dmalloc(&tmp, need ? need : 1));
    WSP_ISTEP(hipcub::DeviceScan::ExclusiveSum(tmp, need, cnt, pad0, (int)(U + 1), s));
    int64_t Rp = 0;
    WSP_ISTEP(hipMemcpyAsync(&Rp, pad0 + U, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    WSP_ISTEP(hipStreamSynchronize(s));
    if (Rp >= 0x7FFFFFC0LL) {  // slots are int32
        cleanup();
        return hipErrorInvalidValue;
    }
    const int64_t n_groups = Rp / 64;
    pl.n_runs_padded = Rp;
    WSP_ISTEP(dalloc(&pl.runrec, Rp));
    WSP_ISTEP(dalloc(&pl.len16, Rp));
    WSP_ISTEP(dalloc(&pl.suf, Rp));
    WSP_ISTEP(dalloc(&pl.run_lay, R));
    WSP_ISTEP(dalloc(&pl.grp_tap, n_groups + 1));
    WSP_ISTEP(dalloc(&grp_unit, n_groups));
    WSP_ISTEP(dalloc(&grp_len, n_groups + 1));
    WSP_ISTEP(dalloc(&steps, 1));
    if (Rp > 0) hipLaunchKernelGGL(k_fill_padding, dim3(grid1d(Rp, 256)), dim3(256), 0, s, Rp, pl.runrec);
    WSP_ISTEP(hipMemsetAsync(pl.len16, 0, sizeof(uint16_t) * (size_t)Rp, s));
    WSP_ISTEP(hipMemsetAsync(steps, 0, sizeof(unsigned long long), s));
    if (R > 0) {
        hipLaunchKernelGGL(k_pad_scatter, dim3(grid1d(R, 256)), dim3(256), 0, s, key_sorted, lay2gen, pl.unit_run0,
                           pad0, rlen, rent, pl.ent, R, pl.tile_band_rows, pl.run_lay, pl.len16, pl.runrec,
                           grp_unit);
    }
    hipLaunchKernelGGL(k_group_sums, dim3(grid1d(n_groups + 1, 256)), dim3(256), 0, s, pl.len16, n_groups,
                       pl.suf, grp_len, steps);
    WSP_ISTEP(hipGetLastError());
    size_t need2 = 0;
    WSP_ISTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, need2, grp_len, pl.grp_tap, (int)(n_groups + 1), s));
    if (need2 > need) {
        dfree(tmp);
        tmp = nullptr;
        WSP_ISTEP(dmalloc(&tmp, need2));
    }
    WSP_ISTEP(hipcub::DeviceScan::ExclusiveSum(tmp, need2, grp_len, pl.grp_tap, (int)(n_groups + 1), s));
    hipLaunchKernelGGL(k_unit_taps_padded, dim3(grid1d(U + 1, 256)), dim3(256), 0, s, pad0, pl.grp_tap, U,
                       pl.unit_tap0, pl.unit_run0);
    if (n_groups > 0) {
        hipLaunchKernelGGL(k_group_bases, dim3(grid1d(n_groups * 64, 256)), dim3(256), 0, s, pl.grp_tap,
                           pl.unit_tap0, grp_unit, n_groups, pl.runrec);
    }
    WSP_ISTEP(hipGetLastError());
    int64_t total = 0;
    unsigned long long st = 0;
    WSP_ISTEP(hipMemcpyAsync(&total, pl.grp_tap + n_groups, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    WSP_ISTEP(hipMemcpyAsync(&st, steps, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    WSP_ISTEP(hipStreamSynchronize(s));  // before the temporaries are released
    pl.group_steps = (int64_t)st;
    cleanup();
    return total == pl.total_taps ? hipSuccess : hipErrorUnknown;  // every tap in exactly one run
#undef WSP_ISTEP
}

// Runs and the band-major tap layout (see Plan), after the work lists.
static hipError_t make_runs(Plan &pl, hipStream_t s) {
    const int64_t E = pl.n_entries;
    const int br = pl.tile_band_rows;
    const int64_t U = (int64_t)pl.n_items * pl.tile_bands;
    int32_t *pos_of = nullptr, *marks = nullptr, *item_of_pos = nullptr, *gidx = nullptr,
            *lay2gen = nullptr, *rlen = nullptr, *rent = nullptr, *pad_cnt = nullptr, *grp_unit = nullptr;
    uint64_t *key = nullptr, *key_sorted = nullptr;
    int64_t *len_lay = nullptr, *start_lay = nullptr, *grp_len = nullptr;
    unsigned long long *steps = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() {
        void *ptrs[] = {pos_of, marks,   item_of_pos, gidx,     lay2gen, rlen, rent,  pad_cnt,
                        grp_unit, key, key_sorted, len_lay, start_lay, grp_len, steps, tmp};
        for (void *q : ptrs) dfree(q);
    };
#define WSP_RSTEP(expr)        \
    do {                       \
        e = (expr);            \
        if (e != hipSuccess) { \
            cleanup();         \
            return e;          \
        }                      \
    } while (0)
    auto scratch = [&](size_t need) -> hipError_t {
        if (need <= tmp_bytes && tmp) return hipSuccess;
        dfree(tmp);
        tmp = nullptr;
        tmp_bytes = need;
        return dmalloc(&tmp, need ? need : 1);
    };
    size_t need = 0;
    // runs per entry, and each entry's first run (generation order)
    int32_t *cnt = nullptr;
    WSP_RSTEP(dalloc(&cnt, E + 1));
    marks = cnt;  // released by cleanup
    WSP_RSTEP(dalloc(&pl.run_first, E + 1));
    hipLaunchKernelGGL(k_run_counts, dim3(grid1d(E + 1, 256)), dim3(256), 0, s, pl.ent, E, br, cnt);
    WSP_RSTEP(hipGetLastError());
    WSP_RSTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, need, cnt, pl.run_first, (int)(E + 1), s));
    WSP_RSTEP(scratch(need));
    WSP_RSTEP(hipcub::DeviceScan::ExclusiveSum(tmp, need, cnt, pl.run_first, (int)(E + 1), s));
    int32_t R32 = 0;
    WSP_RSTEP(hipMemcpyAsync(&R32, pl.run_first + E, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    WSP_RSTEP(hipStreamSynchronize(s));
    const int64_t R = R32;
    pl.n_runs = R;
    pl.n_runs_padded = R;
    pl.group_steps = 0;
    // work position of each entry, item of each work position
    WSP_RSTEP(dalloc(&pos_of, E));
    WSP_RSTEP(dalloc(&item_of_pos, E));
    hipLaunchKernelGGL(k_pos_of, dim3(grid1d(E, 256)), dim3(256), 0, s, pl.ent_sorted, E, pos_of);
    WSP_RSTEP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)(E + 1), s));
    hipLaunchKernelGGL(k_item_marks, dim3(grid1d(pl.n_items, 256)), dim3(256), 0, s, pl.item_start, pl.n_items,
                       cnt);
    WSP_RSTEP(hipGetLastError());
    need = 0;
    WSP_RSTEP(hipcub::DeviceScan::InclusiveSum(nullptr, need, cnt, item_of_pos, (int)E, s));
    WSP_RSTEP(scratch(need));
    WSP_RSTEP(hipcub::DeviceScan::InclusiveSum(tmp, need, cnt, item_of_pos, (int)E, s));
    // runs in generation order, sorted into layout order
    WSP_RSTEP(dalloc(&key, R));
    WSP_RSTEP(dalloc(&key_sorted, R));
    WSP_RSTEP(dalloc(&gidx, R));
    WSP_RSTEP(dalloc(&lay2gen, R));
    WSP_RSTEP(dalloc(&rlen, R));
    WSP_RSTEP(dalloc(&rent, R));
    hipLaunchKernelGGL(k_run_keys, dim3(grid1d(E, 256)), dim3(256), 0, s, pl.ent, pl.run_first, pos_of,
                       item_of_pos, E, br, key, gidx, rlen, rent);
    WSP_RSTEP(hipGetLastError());
    int item_bits = 1;
    while (((int64_t)1 << item_bits) < (int64_t)pl.n_items) ++item_bits;
    if (32 + item_bits > 64) {
        cleanup();
        return hipErrorInvalidValue;
    }
    need = 0;
    WSP_RSTEP(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key, key_sorted, gidx, lay2gen, (int)R, 0,
                                                 32 + item_bits, s));
    WSP_RSTEP(scratch(need));
    WSP_RSTEP(hipcub::DeviceRadixSort::SortPairs(tmp, need, key, key_sorted, gidx, lay2gen, (int)R, 0,
                                                 32 + item_bits, s));
    // units (runs in unpadded layout order)
    WSP_RSTEP(dalloc(&pl.unit_run0, U + 1));
    WSP_RSTEP(dalloc(&pl.unit_tap0, U + 1));
    if (R > 0) {
        hipLaunchKernelGGL(k_unit_heads, dim3(grid1d(R, 256)), dim3(256), 0, s, key_sorted, R, U, pl.tile_bands,
                           pl.unit_run0);
    } else {
        WSP_RSTEP(hipMemsetAsync(pl.unit_run0, 0, sizeof(int32_t) * (size_t)(U + 1), s));
    }
    WSP_RSTEP(hipGetLastError());
    pl.interleaved = pl.layout_param == WSP_LAYOUT_INTERLEAVED;
    if (pl.interleaved) {
        e = make_interleaved(pl, R, U, key_sorted, lay2gen, rlen, rent, s);
        cleanup();
        return e;
    }
    // tap offsets in layout order
    WSP_RSTEP(dalloc(&len_lay, R + 1));
    WSP_RSTEP(dalloc(&start_lay, R + 1));
    WSP_RSTEP(dalloc(&pl.run_tap, R));
    hipLaunchKernelGGL(k_run_lengths, dim3(grid1d(R + 1, 256)), dim3(256), 0, s, lay2gen, rlen, R, len_lay);
    WSP_RSTEP(hipGetLastError());
    need = 0;
    WSP_RSTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, need, len_lay, start_lay, (int)(R + 1), s));
    WSP_RSTEP(scratch(need));
    WSP_RSTEP(hipcub::DeviceScan::ExclusiveSum(tmp, need, len_lay, start_lay, (int)(R + 1), s));
    hipLaunchKernelGGL(k_run_taps, dim3(grid1d(R, 256)), dim3(256), 0, s, lay2gen, start_lay, R, pl.run_tap);
    WSP_RSTEP(dalloc(&pl.run_lay, R));
    hipLaunchKernelGGL(k_run_slots, dim3(grid1d(R, 256)), dim3(256), 0, s, lay2gen, R, pl.run_lay);
    hipLaunchKernelGGL(k_unit_taps, dim3(grid1d(U + 1, 256)), dim3(256), 0, s, pl.unit_run0, start_lay, U,
                       pl.unit_tap0);
    WSP_RSTEP(dalloc(&pl.runrec, R));
    hipLaunchKernelGGL(k_run_records, dim3(grid1d(R, 256)), dim3(256), 0, s, key_sorted, lay2gen, start_lay,
                       pl.unit_tap0, rent, pl.ent, R, br, pl.runrec);
    WSP_RSTEP(hipGetLastError());
    // classes: maximal sequences of runs of one shape within a unit (the key
    // holds the unit and the shape)
    {
        int32_t *head = gidx, *incl = rlen;  // both free now
        uint64_t *cls_key = key;
        WSP_RSTEP(dalloc(&pad_cnt, R + 1));   // first run of each class
        int32_t *cls_run0 = pad_cnt;
        if (R > 0) {
            hipLaunchKernelGGL(k_class_heads, dim3(grid1d(R, 256)), dim3(256), 0, s, key_sorted, R, head);
            need = 0;
            WSP_RSTEP(hipcub::DeviceScan::InclusiveSum(nullptr, need, head, incl, (int)R, s));
            WSP_RSTEP(scratch(need));
            WSP_RSTEP(hipcub::DeviceScan::InclusiveSum(tmp, need, head, incl, (int)R, s));
            int32_t nc32 = 0;
            WSP_RSTEP(hipMemcpyAsync(&nc32, incl + R - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            WSP_RSTEP(hipStreamSynchronize(s));
            pl.n_classes = nc32;
            hipLaunchKernelGGL(k_class_first, dim3(grid1d(R, 256)), dim3(256), 0, s, head, incl, key_sorted, R,
                               cls_run0, cls_key);
        } else {
            pl.n_classes = 0;
        }
        WSP_RSTEP(dalloc(&pl.clsrec, pl.n_classes));
        WSP_RSTEP(dalloc(&pl.unit_cls0, U + 1));
        if (pl.n_classes > 0) {
            hipLaunchKernelGGL(k_class_records, dim3(grid1d(pl.n_classes, 256)), dim3(256), 0, s, cls_run0,
                               cls_key, pl.runrec, pl.n_classes, R, pl.clsrec);
            hipLaunchKernelGGL(k_unit_heads, dim3(grid1d(pl.n_classes, 256)), dim3(256), 0, s, cls_key,
                               pl.n_classes, U, pl.tile_bands, pl.unit_cls0);
            WSP_RSTEP(dalloc(&steps, 1));
            unsigned long long *d_long = steps;
            WSP_RSTEP(hipMemsetAsync(d_long, 0, sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_long_taps, dim3(grid1d(pl.n_classes, 256)), dim3(256), 0, s, pl.clsrec,
                               pl.n_classes, d_long);
            unsigned long long h_long = 0;
            WSP_RSTEP(hipMemcpyAsync(&h_long, d_long, sizeof(h_long), hipMemcpyDeviceToHost, s));
            WSP_RSTEP(hipStreamSynchronize(s));
            pl.long_taps = (int64_t)h_long;
        } else {
            WSP_RSTEP(hipMemsetAsync(pl.unit_cls0, 0, sizeof(int32_t) * (size_t)(U + 1), s));
        }
        WSP_RSTEP(hipGetLastError());
        // bands in decreasing order of taps (a stable sort: ties keep band order)
        WSP_RSTEP(dalloc(&pl.unit_order, U));
        if (U > 0) {
            int64_t *sz = nullptr;
            int32_t *ord_in = nullptr;
            e = dalloc(&sz, 2 * U);
            if (e == hipSuccess) e = dalloc(&ord_in, U);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_unit_sizes, dim3(grid1d(U, 256)), dim3(256), 0, s, pl.unit_tap0, U, sz, ord_in);
                need = 0;
                e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, need, sz, sz + U, ord_in, pl.unit_order,
                                                                 (int)U, 0, 40, s);
            }
            if (e == hipSuccess) e = scratch(need);
            if (e == hipSuccess)
                e = hipcub::DeviceRadixSort::SortPairsDescending(tmp, need, sz, sz + U, ord_in, pl.unit_order,
                                                                 (int)U, 0, 40, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            dfree(sz);
            dfree(ord_in);
            WSP_RSTEP(e);
        }
    }
    int64_t total = 0;
    WSP_RSTEP(hipMemcpyAsync(&total, start_lay + R, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    WSP_RSTEP(hipStreamSynchronize(s));  // before the temporaries are released
    cleanup();
    return total == pl.total_taps ? hipSuccess : hipErrorUnknown;  // every tap in exactly one run
#undef WSP_RSTEP
}

hipError_t make_plan(wsp_ctx *c, const double *d_centres, hipStream_t s, int *support_err) {
    Plan &pl = c->plan;
    const Geom &g = c->g;
    const int64_t m = pl.m;
    *support_err = 0;
    free_sorted_plan(pl);

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
        dfree(t.ux);
        dfree(t.vx);
        dfree(t.weff);
        dfree(t.jp);
        dfree(t.u0w);
        dfree(t.v0w);
        dfree(t.key);
        dfree(key_sorted);
        dfree(cost);
        dfree(cost_sorted);
        dfree(iota);
        dfree(order_tmp);
        dfree(cnt);
        dfree(d_err);
        dfree(tmp);
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
    WSP_STEP(dmalloc(&tmp, tmp_bytes));
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, t.key, key_sorted, iota, pl.perm,
                                                (int)m, 0, key_bits > 0 ? key_bits : 1, s));
    dfree(tmp);
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
    WSP_STEP(dalloc(&pl.iperm, m));
    dim3 gb(grid1d(m, 256)), bb(256);
    hipLaunchKernelGGL(k_invert, gb, bb, 0, s, pl.perm, pl.iperm, m);
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
    WSP_STEP(dmalloc(&tmp, tmp_bytes));
    WSP_STEP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, pl.tap_off, (int)(m + 1), s));
    dfree(tmp);
    tmp = nullptr;
    hipLaunchKernelGGL(k_iota, dim3(grid1d(m, 256)), dim3(256), 0, s, iota, m);
    tmp_bytes = 0;
    WSP_STEP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, cost, cost_sorted, iota,
                                                pl.border, (int)m, 0, 32, s));
    WSP_STEP(dmalloc(&tmp, tmp_bytes));
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
    pl.tile_bits = tile_bits;
    cleanup();
    if (g.planes) {
        // the lattice layout sets the bands of the work order
        bool too_large = false;
        hipError_t e2 = plane_layout(c, s, &too_large);
        if (e2 != hipSuccess) return e2;
        if (too_large) {
            *support_err |= 4;
            return hipSuccess;
        }
    }
    hipError_t e3 = make_entries(pl, g, tile_bits, s);
    if (e3 != hipSuccess || g.planes) return e3;
    // bands of 8 rows unless asked otherwise (16-row bands halve the run
    // kernels' occupancy, which costs more than the longer runs gain)
    pl.tile_band_rows = g.band_rows_param > 0 ? g.band_rows_param : 8;
    pl.tile_bands = kTile / pl.tile_band_rows;
    pl.layout_param = g.tap_layout_param;
    if (pl.n_entries >= 0x7FFFFFF0LL / pl.tile_bands) return hipErrorInvalidValue;  // run indices are int32
    return make_runs(pl, s);
#undef WSP_STEP
}

}  // namespace wsp
