// Operator application: y = Phi x (degrid) and x = Re Phi^dagger y (grid),
// Eqs. (2)-(7).  Per stack k:
//   degrid: S~_k and Z (k_taper_half), F (batched 1-D hipFFT passes with
//           k_transpose_pad between them), GC_k and W_k (k_degrid_tiles or
//           k_degrid_small, then k_degrid_reduce);
//   grid:   W_k (k_prep_vis), GC_k^dagger (k_grid_tiles or k_grid_small,
//           then k_reduce_tiles), F^dagger (hipFFT passes with
//           k_transpose_crop), Z^dagger, S~_k^dagger, Re and the sum over
//           stacks (k_crop_half).
// Both sparse steps work on the tile work lists of the plan: each work item
// is a run of (visibility, 64 x 64 grid tile) entries of one tile.
#include <type_traits>

#include "wsp_devmath.h"
#include "wsp_image.h"
#include "wsp_plane.h"

namespace wsp {

namespace {

// F is computed in two passes of batched 1-D transforms of length G, with the
// data transposed in between, so that neither pass touches the zero padding
// that Z adds or the cells that Z^dagger discards:
//   forward: H[k][i][V] = z_k[V][U(i)] for the N padded-image columns U(i)
//            that hold pixels (k_taper_half), transform along V (rows of H),
//            transpose into the grid with zero columns elsewhere
//            (k_transpose_pad), transform along U (rows of the grid);
//   inverse: transform along U, keep the N columns U(i) that the crop
//            needs, transposed into H (k_transpose_crop), transform along V,
//            crop, untaper and sum over stacks (k_crop_half).
// Each transposing kernel stages a 64 x 64 tile in LDS so that its reads and
// writes are both coalesced.
constexpr int kT = 64;

// S~_k and Z for all stacks, written as H.  Block: (V tile, pixel-column tile).
template <bool kFP64>
__global__ __launch_bounds__(256) void k_taper_half(const typename Types<kFP64>::R *__restrict__ image,
                                                    typename Types<kFP64>::C *half,
                                                    const double *__restrict__ centres, Geom g) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ R s_x[kT][kT + 1];  // [V offset][i offset]
    const int V0 = blockIdx.x * kT, i0 = blockIdx.y * kT;
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int r = e / kT, cc = e % kT;  // along i: coalesced image reads
        const int j = pixel_of(V0 + r, g), i = i0 + cc;
        s_x[r][cc] = (j >= 0 && i < g.n) ? image[(int64_t)j * g.n + i] : (R)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int cc = e / kT, r = e % kT;  // along V: coalesced writes of H
        const int i = i0 + cc, V = V0 + r;
        if (i >= g.n) continue;
        const int j = pixel_of(V, g);
        C z;
        z.x = 0;
        z.y = 0;
        if (j < 0) {
            for (int k = 0; k < g.n_stacks; ++k) half[((int64_t)k * g.n + i) * g.G + V] = z;
            continue;
        }
        double amp, nm1;
        pixel_factors(j, i, g, &amp, &nm1);
        const R a = (R)((double)s_x[r][cc] * amp);
        for (int k = 0; k < g.n_stacks; ++k) {
            R sn, cs;
            rev_sincos<kFP64>(reduce_rev(-centres[k] * nm1), &sn, &cs);
            z.x = a * cs;
            z.y = a * sn;
            half[((int64_t)k * g.n + i) * g.G + V] = z;
        }
    }
}

// grid[k][V][U] = H[k][i][V] where U = U(i), else 0.  Block: (V tile, U tile, stack).
template <typename C>
__global__ __launch_bounds__(256) void k_transpose_pad(const C *__restrict__ half, C *grids, Geom g) {
    __shared__ C s_t[kT][kT + 1];  // [U offset][V offset]
    const int V0 = blockIdx.x * kT, U0 = blockIdx.y * kT, k = blockIdx.z;
    if (!row_used(V0, g)) return;  // rows that no work item reads (uniform)
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int u = e / kT, v = e % kT;  // along V: coalesced reads of H
        const int i = pixel_of(U0 + u, g);
        C z;
        z.x = 0;
        z.y = 0;
        if (i >= 0) z = half[((int64_t)k * g.n + i) * g.G + V0 + v];
        s_t[u][v] = z;
    }
    __syncthreads();
    C *dst = grids + (int64_t)k * g.G * g.G;
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int v = e / kT, u = e % kT;  // along U: coalesced grid writes
        dst[(int64_t)(V0 + v) * g.G + U0 + u] = s_t[u][v];
    }
}

// H[k][i][V] = grid[k][V][U(i)] for the N pixel columns.  Block: (V tile, i tile, stack).
template <typename C>
__global__ __launch_bounds__(256) void k_transpose_crop(const C *__restrict__ grids, C *half, Geom g) {
    __shared__ C s_t[kT][kT + 1];  // [V offset][i offset]
    const int V0 = blockIdx.x * kT, i0 = blockIdx.y * kT, k = blockIdx.z;
    const C *src = grids + (int64_t)k * g.G * g.G;
    const bool used = row_used(V0, g);  // rows without work items hold zeros (uniform)
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int v = e / kT, cc = e % kT;  // along i (U): coalesced grid reads
        const int i = i0 + cc;
        C z;
        z.x = 0;
        z.y = 0;
        if (used && i < g.n) z = src[(int64_t)(V0 + v) * g.G + padded_of(i, g)];
        s_t[v][cc] = z;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int cc = e / kT, v = e % kT;  // along V: coalesced writes of H
        const int i = i0 + cc;
        if (i < g.n) half[((int64_t)k * g.n + i) * g.G + V0 + v] = s_t[v][cc];
    }
}

// Z^dagger, S~_k^dagger, Re and the sum over stacks from H.  Block: (j tile, i tile).
template <bool kFP64>
__global__ __launch_bounds__(256) void k_crop_half(const typename Types<kFP64>::C *__restrict__ half,
                                                   typename Types<kFP64>::R *image,
                                                   const double *__restrict__ centres, Geom g) {
    using R = typename Types<kFP64>::R;
    __shared__ R s_o[kT][kT + 1];  // [i offset][j offset]
    const int j0 = blockIdx.x * kT, i0 = blockIdx.y * kT;
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int cc = e / kT, r = e % kT;  // along j (V): coalesced reads of H
        const int i = i0 + cc, j = j0 + r;
        R out = 0;
        if (i < g.n && j < g.n) {
            const int V = padded_of(j, g);
            double amp, nm1;
            pixel_factors(j, i, g, &amp, &nm1);
            double acc = 0.0;
            for (int k = 0; k < g.n_stacks; ++k) {
                R sn, cs;
                rev_sincos<kFP64>(reduce_rev(-centres[k] * nm1), &sn, &cs);
                const auto z = half[((int64_t)k * g.n + i) * g.G + V];
                // Re(z conj(s_k)) with s_k = amp e^{2 pi i rev}
                acc += (double)(z.x * cs + z.y * sn);
            }
            out = (R)(amp * acc);
        }
        s_o[cc][r] = out;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
        const int r = e / kT, cc = e % kT;  // along i: coalesced image writes
        const int i = i0 + cc, j = j0 + r;
        if (i < g.n && j < g.n) image[(int64_t)j * g.n + i] = s_o[cc][r];
    }
}

// Zero the used rows of the grids (the others are never read).
template <typename C>
__global__ void k_zero_rows(C *grids, Geom g) {
    const int rows = g.rows_lo + g.rows_hi;
    const int64_t n = (int64_t)g.n_stacks * rows * g.G;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t kr = i / g.G;
    const int U = (int)(i - kr * g.G);
    const int k = (int)(kr / rows), r = (int)(kr - (int64_t)k * rows);
    const int V = r < g.rows_lo ? r : g.G - g.rows_hi + (r - g.rows_lo);
    C z;
    z.x = 0;
    z.y = 0;
    grids[((int64_t)k * g.G + V) * g.G + U] = z;
}

struct ApplyArgs {
    const int32_t *perm, *jp, *u0w, *v0w, *stack;
    const double *wt;
    const uint8_t *sflag;
    const int32_t *iperm;      // caller -> sorted
    const double *wt_in;       // caller order
    const uint8_t *flag;       // caller order
    const int64_t *tap_off;
    int64_t m;
    Geom g;
};

template <typename R>
__device__ __forceinline__ R wave_sum_r(R x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// W_k and Eq. (8) on the adjoint's input: yw[p] = W_p (conj) y[perm[p]] in
// sorted order.  rot = 1 takes -i y instead (the Stokes U half of the
// polarised adjoint, Eq. (9)).  One thread per caller-order visibility:
// its reads are coalesced and only the store is scattered (a gather in
// sorted order would fetch a cache line per 8-byte visibility).
template <bool kFP64>
__global__ void k_prep_vis(const typename Types<kFP64>::C *__restrict__ vis,
                           typename Types<kFP64>::C *yw, ApplyArgs a, int rot) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.m) return;
    C y = vis[q];
    if (rot) {
        const R re = y.x;
        y.x = y.y;
        y.y = -re;
    }
    R w = (R)a.wt_in[q];
    C o;
    o.x = y.x * w;
    o.y = (a.flag[q] ? -y.y : y.y) * w;
    yw[a.iperm[q]] = o;
}

struct TileArgs {
    const int4 *wrec;           // entry records in work-list order
    const int32_t *ent_sorted;  // entry indices in work-list order
    const int32_t *item_start;
    const uint32_t *item_key;
    const uint8_t *item_sole;
    const int32_t *item_slot;
    void *partial;
    int n_items;
    int tile_bits;
    int G;
    const int32_t *itile;       // items grouped by tile (for the split-tile reduction)
    // w-plane mode: per-entry plane records (work-list order) and the lattice
    const int4 *prec;
    const float *ptw;
    const float4 *table;
    float inv_dq;
};

// XCD-aware block order: consecutive items (neighbouring tiles) go to the
// same XCD, which dispatches blocks round-robin over its 8 dies.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int nx = 8;
    int per = (n + nx - 1) / nx;
    return (b % nx) * per + b / nx;
}

// The same for kH blocks per item: the blocks of an item go to one XCD (8
// block indices apart), so rows of an entry split between them share that
// XCD's L2.  *part = which block of the item.
__device__ __forceinline__ int xcd_item_part(int b, int n, int kH, int *part) {
    const int nx = 8;
    const int r = b / nx;
    *part = r % kH;
    const int per = (n + nx - 1) / nx;
    return (b % nx) * per + r / kH;
}

// First cell of a (stack, tile) key in the grids.
template <typename C>
__device__ __forceinline__ C *tile_origin(C *grids, uint32_t key, int tile_bits, int G) {
    const int tmask = (1 << tile_bits) - 1;
    const int tx = key & tmask, ty = (key >> tile_bits) & tmask;
    const int k = key >> (2 * tile_bits);
    return grids + (int64_t)k * G * G + (int64_t)ty * kTile * G + (int64_t)tx * kTile;
}
template <typename C>
__device__ __forceinline__ C *tile_origin(C *grids, uint32_t key, const TileArgs &t) {
    return tile_origin(grids, key, t.tile_bits, t.G);
}

constexpr int kWaves = 8;             // wavefronts per block of the tile kernels
constexpr int kThreads = 64 * kWaves;
constexpr int kChunk = 256;           // degrid: entries whose metadata is staged in LDS at a time
constexpr int kGChunk = 128;          // grid: the same (smaller: the block also holds y per entry)
constexpr int kBand = kTile / kWaves; // grid: tile rows owned by each wavefront
constexpr int64_t kSmallEntryTaps = 160;  // mean taps per entry below which k_degrid_small / k_grid_small run
// grid: blocks per work item, each owning kTile / split rows of the tile (more,
// smaller blocks keep more wavefronts resident when bands finish unevenly)
constexpr int kGridSplit = 2;
constexpr int kGridSplitSmall = 4;

typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef double v2d_t __attribute__((ext_vector_type(2)));

// Tap loads: every tap is read once per operator application, so they are
// issued non-temporal and do not evict reused data (the staged grid tiles)
// from the caches.
__device__ __forceinline__ float2 load_tap(const float2 *p) {
    const v2f_t t = __builtin_nontemporal_load((const v2f_t *)p);
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ double2 load_tap(const double2 *p) {
    const v2d_t t = __builtin_nontemporal_load((const v2d_t *)p);
    return make_double2(t.x, t.y);
}

// Row and column of tap k in a row-major sub-block nc wide.  (k + 1/2) / nc
// is never within 1/(2 nc) of an integer, and (k + 1/2) * rcp(nc) with the
// hardware reciprocal (1 ulp) is off by < 4096 * 2.4e-7 < 1/128 <= 1/(2 nc),
// so the row is exact; both products fit the 24-bit multiplier.
__device__ __forceinline__ float recip_nc(int nc) { return __builtin_amdgcn_rcpf((float)nc); }
__device__ __forceinline__ int sub_row(int k, float inv_nc) { return (int)(((float)k + 0.5f) * inv_nc); }
__device__ __forceinline__ int sub_cell(int cell0, int k, int row, int nc) {
    return cell0 + row * kTile + (k - (int)__umul24((unsigned)row, (unsigned)nc));
}

// The wavefront's index in its block, known to the compiler as uniform over
// the wavefront (so that everything derived from it stays in scalar registers
// and scalar branches).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// value of lane l (l uniform over the wavefront)
__device__ __forceinline__ float bcast(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double bcast(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Batches of U x 64 consecutive taps of a run: 8 while at least 6 blocks of
// 64 taps are left, then 4, 2, 1, so a run's tail issues few redundant loads
// and the bulk keeps 8 loads per lane in flight.  kWide (w-plane kernels,
// whose lattice lookups are latency-bound) adds batches of 16 while at least
// 12 blocks are left.
template <bool kWide = false, typename F>
__device__ __forceinline__ void for_batches(int kbeg, int kend, F &&f) {
    for (int k0 = kbeg; k0 < kend;) {
        const int nb = (kend - k0 + 63) >> 6;  // uniform over the wavefront
        if (kWide && nb >= 12) {
            f(k0, std::integral_constant<int, 16>());
            k0 += 1024;
        } else if (nb >= 6) {
            f(k0, std::integral_constant<int, 8>());
            k0 += 512;
        } else if (nb >= 3) {
            f(k0, std::integral_constant<int, 4>());
            k0 += 256;
        } else if (nb == 2) {
            f(k0, std::integral_constant<int, 2>());
            k0 += 128;
        } else {
            f(k0, std::integral_constant<int, 1>());
            k0 += 64;
        }
    }
}

// GC_k, W_k (degrid), one block per work item: the item's 64 x 64 grid tile
// is staged in LDS; the wavefronts take entries in turn, lanes walk the
// entry's tap sub-block, multiply by the staged grid values and reduce; each
// entry's partial sum goes to dpart[entry] (entries are stored grouped by
// visibility), summed per visibility by k_degrid_reduce.
template <bool kFP64, bool kPlanes>
__global__ __launch_bounds__(kThreads) void k_degrid_tiles(const typename Types<kFP64>::C *__restrict__ taps,
                                                           const typename Types<kFP64>::C *__restrict__ grids,
                                                           typename Types<kFP64>::C *dpart, TileArgs t) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ C tile[kTile * kTile];
    __shared__ int s_geo[kChunk];  // nc | nr << 8 | lx0 << 16 | ly0 << 24
    __shared__ int s_idx[kChunk];
    __shared__ int64_t s_off[kPlanes ? 1 : kChunk];
    __shared__ int4 s_prec[kPlanes ? kChunk : 1];
    __shared__ float s_sw[kPlanes ? kChunk : 1];
    const int item = xcd_item(blockIdx.x, t.n_items);
    if (item >= t.n_items) return;  // uniform over the block
    {
        const C *src = tile_origin(grids, t.item_key[item], t);
        for (int i = threadIdx.x; i < kTile * kTile; i += kThreads)
            tile[i] = src[(int64_t)(i / kTile) * t.G + (i % kTile)];
    }
    const int lane = threadIdx.x & 63;
    const int wid = wave_index();
    const int s_beg = t.item_start[item], s_end = t.item_start[item + 1];
    for (int base = s_beg; base < s_end; base += kChunk) {
        const int n = (s_end - base < kChunk) ? s_end - base : kChunk;
        __syncthreads();  // tile staged / previous chunk consumed
        for (int q = threadIdx.x; q < n; q += kThreads) {
            const int4 rec = t.wrec[base + q];
            s_geo[q] = rec.z;
            s_idx[q] = t.ent_sorted[base + q];
            if constexpr (kPlanes) {
                s_prec[q] = t.prec[base + q];
                s_sw[q] = t.ptw[base + q];
            } else {
                s_off[q] = ((int64_t)rec.y << 32) | (uint32_t)rec.x;
            }
        }
        __syncthreads();
        for (int j = wid; j < n; j += kWaves) {
            const int geo = s_geo[j];
            const int nc = geo & 255, nr = (geo >> 8) & 255;
            const int lx0 = (geo >> 16) & 255, ly0 = (geo >> 24) & 255;
            const C *tp = taps;
            PlaneEntry pe{};
            if constexpr (kPlanes) pe = plane_entry(s_prec[j], s_sw[j], t.table);
            else tp = taps + s_off[j];
            const float inv_nc = recip_nc(nc);
            const int ntap = nr * nc;
            const int cell0 = ly0 * kTile + lx0;  // tile cell of sub-block tap 0
            R ar = 0, ai = 0;
            for_batches<kPlanes>(0, ntap, [&](int k0, auto ucount) {
                constexpr int U = decltype(ucount)::value;
                C K[U];
                int li[U];
                PlaneLoad L[kPlanes ? U : 1];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // past the sub-block: re-read tap 0 and weight it by zero below
                    const int k = k0 + 64 * u + lane < ntap ? k0 + 64 * u + lane : 0;
                    const int row = sub_row(k, inv_nc);
                    li[u] = sub_cell(cell0, k, row, nc);
                    if constexpr (kPlanes) L[u] = plane_load(pe, row, k - (int)__umul24((unsigned)row, (unsigned)nc), t.inv_dq);
                    else K[u] = load_tap(&tp[k]);  // the sub-block is contiguous, row-major
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if constexpr (kPlanes) {
                        const float2 v = plane_value(L[u], pe.sw, pe.sgn);
                        K[u].x = v.x;
                        K[u].y = v.y;
                    }
                    const bool ok = k0 + 64 * u + lane < ntap;
                    const C z = tile[li[u]];
                    const R kr = ok ? K[u].x : (R)0, ki = ok ? K[u].y : (R)0;
                    ar += kr * z.x - ki * z.y;
                    ai += kr * z.y + ki * z.x;
                }
            });
            ar = wave_sum_r(ar);
            ai = wave_sum_r(ai);
            if (lane == 0) {
                C o;
                o.x = ar;
                o.y = ai;
                dpart[s_idx[j]] = o;
            }
        }
    }
}

// Degrid for work lists of small entries (a few tens of taps, as with many
// w-stacks): 16-lane groups take one entry each, so a wavefront reduces 4
// entries per pass instead of spreading one entry over 64 lanes.  Otherwise
// as k_degrid_tiles.
constexpr int kGroup = 16;
template <bool kFP64, bool kPlanes>
__global__ __launch_bounds__(kThreads) void k_degrid_small(const typename Types<kFP64>::C *__restrict__ taps,
                                                           const typename Types<kFP64>::C *__restrict__ grids,
                                                           typename Types<kFP64>::C *dpart, TileArgs t) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int kPer = 64 / kGroup;  // entries per wavefront pass
    // load slots per lane; w-plane kernels use 4 (their lookups hit a
    // cache-resident lattice, and the extra resident wavefronts hide more)
    constexpr int kU = kPlanes ? 4 : 8;
    __shared__ C tile[kTile * kTile];
    __shared__ int s_geo[kChunk];  // nc | nr << 8 | lx0 << 16 | ly0 << 24
    __shared__ int s_idx[kChunk];
    __shared__ int64_t s_off[kPlanes ? 1 : kChunk];
    __shared__ int4 s_prec[kPlanes ? kChunk : 1];
    __shared__ float s_sw[kPlanes ? kChunk : 1];
    const int item = xcd_item(blockIdx.x, t.n_items);
    if (item >= t.n_items) return;  // uniform over the block
    {
        const C *src = tile_origin(grids, t.item_key[item], t);
        for (int i = threadIdx.x; i < kTile * kTile; i += kThreads)
            tile[i] = src[(int64_t)(i / kTile) * t.G + (i % kTile)];
    }
    const int lane = threadIdx.x & 63;
    const int wid = wave_index();
    const int grp = lane / kGroup, gl = lane % kGroup;
    const int s_beg = t.item_start[item], s_end = t.item_start[item + 1];
    for (int base = s_beg; base < s_end; base += kChunk) {
        const int n = (s_end - base < kChunk) ? s_end - base : kChunk;
        __syncthreads();  // tile staged / previous chunk consumed
        for (int q = threadIdx.x; q < n; q += kThreads) {
            const int4 rec = t.wrec[base + q];
            s_geo[q] = rec.z;
            s_idx[q] = t.ent_sorted[base + q];
            if constexpr (kPlanes) {
                s_prec[q] = t.prec[base + q];
                s_sw[q] = t.ptw[base + q];
            } else {
                s_off[q] = ((int64_t)rec.y << 32) | (uint32_t)rec.x;
            }
        }
        __syncthreads();
        for (int j0 = wid * kPer; j0 < n; j0 += kWaves * kPer) {
            const int j = j0 + grp;
            const bool valid = j < n;
            const int geo = s_geo[valid ? j : j0];
            const int nc = geo & 255, nr = (geo >> 8) & 255;
            const int lx0 = (geo >> 16) & 255, ly0 = (geo >> 24) & 255;
            const C *tp = taps;
            PlaneEntry pe{};
            if constexpr (kPlanes) pe = plane_entry(s_prec[valid ? j : j0], s_sw[valid ? j : j0], t.table);
            else tp = taps + s_off[valid ? j : j0];
            const float inv_nc = recip_nc(nc);
            const int ntap = valid ? nr * nc : 0;
            const int cell0 = ly0 * kTile + lx0;
            R ar = 0, ai = 0;
            for (int k0 = 0; __any(k0 < ntap); k0 += kGroup * kU) {
                C K[kU];
                int li[kU];
                PlaneLoad L[kPlanes ? kU : 1];
                // slots past every group's entry are skipped (uniform), lanes past
                // their own entry load nothing and add zero
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    K[u].x = 0;
                    K[u].y = 0;
                    if constexpr (kPlanes) L[u] = plane_zero();
                    li[u] = cell0;
                    const bool ok = k0 + kGroup * u + gl < ntap;
                    if (__any(ok)) {
                        const int k = ok ? k0 + kGroup * u + gl : 0;
                        const int row = sub_row(k, inv_nc);
                        li[u] = sub_cell(cell0, k, row, nc);
                        if (ok) {
                            if constexpr (kPlanes) L[u] = plane_load(pe, row, k - (int)__umul24((unsigned)row, (unsigned)nc), t.inv_dq);
                            else K[u] = load_tap(&tp[k]);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if constexpr (kPlanes) {
                        const float2 v = plane_value(L[u], pe.sw, pe.sgn);
                        K[u].x = v.x;
                        K[u].y = v.y;
                    }
                    const bool ok = k0 + kGroup * u + gl < ntap;
                    const C z = tile[li[u]];
                    const R kr = ok ? K[u].x : (R)0, ki = ok ? K[u].y : (R)0;
                    ar += kr * z.x - ki * z.y;
                    ai += kr * z.y + ki * z.x;
                }
            }
            // sum over the 16 lanes of the group
#pragma unroll
            for (int o = kGroup / 2; o > 0; o >>= 1) {
                ar += __shfl_xor(ar, o, 64);
                ai += __shfl_xor(ai, o, 64);
            }
            if (gl == 0 && valid) {
                C o;
                o.x = ar;
                o.y = ai;
                dpart[s_idx[j]] = o;
            }
        }
    }
}

// y[perm[p]] = W_p (conj) sum of visibility p's entry partials, in entry order.
// add_i = 1 adds i times that value to y[perm[p]] instead (the Stokes U half
// of the polarised degrid: each Stokes image is folded on its own, Eq. (9)).
template <bool kFP64>
__global__ void k_degrid_reduce(const typename Types<kFP64>::C *__restrict__ dpart,
                                const int64_t *__restrict__ ent_off,
                                typename Types<kFP64>::C *vis, ApplyArgs a, int add_i) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.m) return;
    R ar = 0, ai = 0;
    for (int64_t e = ent_off[p]; e < ent_off[p + 1]; ++e) {
        C v = dpart[e];
        ar += v.x;
        ai += v.y;
    }
    R w = (R)a.wt[p];
    C y;
    y.x = ar * w;
    y.y = (a.sflag[p] ? -ai : ai) * w;  // Eq. (8): folded visibilities are conjugated
    if (add_i) {
        C o = vis[a.perm[p]];
        o.x -= y.y;
        o.y += y.x;
        y = o;
    }
    vis[a.perm[p]] = y;
}

// GC_k^dagger (grid), kH blocks per work item, no atomics: block b of an item
// accumulates rows [64 b / kH, 64 (b + 1) / kH) of the item's 64 x 64 tile in
// LDS, and each of its wavefronts owns 8 of those rows: no other wavefront
// touches them.  Every wavefront scans all entries of the
// item (64 per ballot); for each entry with rows in its band it streams the
// taps of those rows (a contiguous run of the row-major sub-block), lanes on
// consecutive taps, and adds conj(K) yw to the owned cells.  The cells of one entry are distinct
// and a wavefront's LDS accesses complete in order, so plain read-modify-
// write is exact.  The tile is then stored into the grid (the tile's only
// item) or into a partial-tile slot that k_reduce_tiles sums in item order.
template <bool kFP64, int kH, bool kPlanes>
__global__ __launch_bounds__(kThreads / kH, kFP64 ? 4 : 8) void k_grid_tiles(const typename Types<kFP64>::C *__restrict__ taps,
                                                         const typename Types<kFP64>::C *__restrict__ yw,
                                                         typename Types<kFP64>::C *grids, TileArgs t) {
    using C = typename Types<kFP64>::C;
    constexpr int kRows = kTile / kH;  // tile rows of this block
    __shared__ C tile[kRows * kTile + 1];  // + a spare cell for lanes without a tap
    __shared__ int s_geo[kGChunk];  // nc | nr << 8 | lx0 << 16 | ly0 << 24
    __shared__ int64_t s_off[kPlanes ? 1 : kGChunk];
    __shared__ int4 s_prec[kPlanes ? kGChunk : 1];
    __shared__ float s_sw[kPlanes ? kGChunk : 1];
    __shared__ C s_y[kGChunk];
    static_assert(kGChunk <= kThreads / kH, "one thread stages one entry");
    int part;
    const int item = xcd_item_part(blockIdx.x, t.n_items, kH, &part);
    if (item >= t.n_items) return;  // uniform over the block
    const int lane = threadIdx.x & 63;
    const int lrow0 = wave_index() * kBand;  // band start in the LDS tile
    const int band0 = part * kRows + lrow0;       // and in the grid tile
    C zero;
    zero.x = 0;
    zero.y = 0;
    for (int i = lane; i < kBand * kTile; i += 64) tile[lrow0 * kTile + i] = zero;
    const int s_beg = t.item_start[item], s_end = t.item_start[item + 1];
    for (int base = s_beg; base < s_end; base += kGChunk) {
        const int n = (s_end - base < kGChunk) ? s_end - base : kGChunk;
        __syncthreads();  // previous chunk consumed
        if ((int)threadIdx.x < n) {
            const int4 rec = t.wrec[base + threadIdx.x];
            s_geo[threadIdx.x] = rec.z;
            if constexpr (kPlanes) {
                s_prec[threadIdx.x] = t.prec[base + threadIdx.x];
                s_sw[threadIdx.x] = t.ptw[base + threadIdx.x];
            } else {
                s_off[threadIdx.x] = ((int64_t)rec.y << 32) | (uint32_t)rec.x;
            }
            s_y[threadIdx.x] = yw[rec.w];
        }
        __syncthreads();
        // 64 entries at a time: lane l holds entry j0 + l; a ballot marks the
        // entries with rows in this band, whose fields are then broadcast
        // with readlane (no memory round trip per entry).
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int jl = j0 + lane;
            int geo_l = 0;
            int64_t off_l = 0;
            int4 prec_l = make_int4(0, 0, 0, 0);
            float sw_l = 0.0f;
            C y_l = zero;
            if (jl < n) {
                geo_l = s_geo[jl];
                if constexpr (kPlanes) {
                    prec_l = s_prec[jl];
                    sw_l = s_sw[jl];
                } else {
                    off_l = s_off[jl];
                }
                y_l = s_y[jl];
            }
            const int nr_l = (geo_l >> 8) & 255, ly0_l = (geo_l >> 24) & 255;
            uint64_t hits = __ballot(jl < n && ly0_l < band0 + kBand && ly0_l + nr_l > band0);
            while (hits) {
                const int l = __builtin_ctzll(hits);
                hits &= hits - 1;
                const int ez = __builtin_amdgcn_readlane(geo_l, l);
                int64_t off = 0;
                PlaneEntry pe{};
                if constexpr (kPlanes) {
                    const int4 pr = make_int4(__builtin_amdgcn_readlane(prec_l.x, l),
                                              __builtin_amdgcn_readlane(prec_l.y, l),
                                              __builtin_amdgcn_readlane(prec_l.z, l),
                                              __builtin_amdgcn_readlane(prec_l.w, l));
                    pe = plane_entry(pr, bcast(sw_l, l), t.table);
                } else {
                    off = ((int64_t)__builtin_amdgcn_readlane((int)(off_l >> 32), l) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)off_l, l);
                }
                C y;
                y.x = bcast(y_l.x, l);
                y.y = bcast(y_l.y, l);
                const int nr = (ez >> 8) & 255, ly0 = (ez >> 24) & 255;
                const int lo = ly0 > band0 ? ly0 : band0;
                const int hi = (ly0 + nr < band0 + kBand) ? ly0 + nr : band0 + kBand;
                const int nc = ez & 255, lx0 = (ez >> 16) & 255;
                const C *tp = taps + off;
                const int kbeg = (lo - ly0) * nc, kend = (hi - ly0) * nc;
                const float inv_nc = recip_nc(nc);
                const int cell0 = (ly0 - part * kRows) * kTile + lx0;  // LDS cell of sub-block tap 0
                for_batches<kPlanes>(kbeg, kend, [&](int k0, auto ucount) {
                    constexpr int U = decltype(ucount)::value;
                    C K[U], z[U];
                    int li[U];
                    PlaneLoad L[kPlanes ? U : 1];
                    // past the run: re-read its first tap and add zero to the spare cell
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool ok = k0 + 64 * u + lane < kend;
                        const int k = ok ? k0 + 64 * u + lane : kbeg;
                        const int row = sub_row(k, inv_nc);
                        li[u] = ok ? sub_cell(cell0, k, row, nc) : kRows * kTile;
                        if constexpr (kPlanes) L[u] = plane_load(pe, row, k - (int)__umul24((unsigned)row, (unsigned)nc), t.inv_dq);
                        else K[u] = load_tap(&tp[k]);
                    }
                    // all reads before all writes: the cells of the U x 64 taps are
                    // distinct (only the spare cell repeats)
#pragma unroll
                    for (int u = 0; u < U; ++u) z[u] = tile[li[u]];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if constexpr (kPlanes) {
                            const float2 v = plane_value(L[u], pe.sw, pe.sgn);
                            K[u].x = v.x;
                            K[u].y = v.y;
                        }
                        const bool ok = k0 + 64 * u + lane < kend;
                        using R = decltype(K[u].x);
                        const R kr = ok ? K[u].x : (R)0, ki = ok ? K[u].y : (R)0;
                        C o;
                        o.x = z[u].x + (kr * y.x + ki * y.y);
                        o.y = z[u].y + (kr * y.y - ki * y.x);
                        tile[li[u]] = o;
                    }
                });
            }
        }
    }
    const uint32_t key = t.item_key[item];
    C *dst;
    int64_t ld;
    if (t.item_sole[item]) {
        dst = tile_origin(grids, key, t);
        ld = t.G;
    } else {
        dst = (C *)t.partial + (int64_t)t.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    // the band was written by this wavefront only: no barrier needed
#pragma unroll
    for (int r = 0; r < kBand; ++r) dst[(int64_t)(band0 + r) * ld + lane] = tile[(lrow0 + r) * kTile + lane];
}

// Grid for work lists of small entries: band ownership, ballot scan and
// tile layout as in k_grid_tiles, but the band runs are short (a few tens of
// taps), so one run per batch would keep one load per lane in flight.  Here
// the loads of up to kSlots consecutive 64-tap slots (from any number of
// runs) are issued together; then the slots are added into the tile one
// after the other, in entry order (two entries may share cells).
constexpr int kSlots = 8;
template <bool kFP64, int kH, bool kPlanes>
__global__ __launch_bounds__(kThreads / kH, kFP64 ? 4 : 8) void k_grid_small(const typename Types<kFP64>::C *__restrict__ taps,
                                                                        const typename Types<kFP64>::C *__restrict__ yw,
                                                                        typename Types<kFP64>::C *grids, TileArgs t) {
    using C = typename Types<kFP64>::C;
    constexpr int kS = kPlanes ? kSlots / 2 : kSlots;  // slots (4 for w-plane kernels, as in degrid)
    constexpr int kRows = kTile / kH;  // tile rows of this block
    __shared__ C tile[kRows * kTile + 1];  // + a spare cell for lanes without a tap
    __shared__ int s_geo[kGChunk];  // nc | nr << 8 | lx0 << 16 | ly0 << 24
    __shared__ int64_t s_off[kPlanes ? 1 : kGChunk];
    __shared__ int4 s_prec[kPlanes ? kGChunk : 1];
    __shared__ float s_sw[kPlanes ? kGChunk : 1];
    __shared__ C s_y[kGChunk];
    int part;
    const int item = xcd_item_part(blockIdx.x, t.n_items, kH, &part);
    if (item >= t.n_items) return;  // uniform over the block
    const int lane = threadIdx.x & 63;
    const int lrow0 = wave_index() * kBand;  // band start in the LDS tile
    const int band0 = part * kRows + lrow0;       // and in the grid tile
    C zero;
    zero.x = 0;
    zero.y = 0;
    for (int i = lane; i < kBand * kTile; i += 64) tile[lrow0 * kTile + i] = zero;
    const int s_beg = t.item_start[item], s_end = t.item_start[item + 1];
    for (int base = s_beg; base < s_end; base += kGChunk) {
        const int n = (s_end - base < kGChunk) ? s_end - base : kGChunk;
        __syncthreads();  // previous chunk consumed
        if ((int)threadIdx.x < n) {
            const int4 rec = t.wrec[base + threadIdx.x];
            s_geo[threadIdx.x] = rec.z;
            if constexpr (kPlanes) {
                s_prec[threadIdx.x] = t.prec[base + threadIdx.x];
                s_sw[threadIdx.x] = t.ptw[base + threadIdx.x];
            } else {
                s_off[threadIdx.x] = ((int64_t)rec.y << 32) | (uint32_t)rec.x;
            }
            s_y[threadIdx.x] = yw[rec.w];
        }
        __syncthreads();
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int jl = j0 + lane;
            int geo_l = 0;
            int64_t off_l = 0;
            int4 prec_l = make_int4(0, 0, 0, 0);
            float sw_l = 0.0f;
            C y_l = zero;
            if (jl < n) {
                geo_l = s_geo[jl];
                if constexpr (kPlanes) {
                    prec_l = s_prec[jl];
                    sw_l = s_sw[jl];
                } else {
                    off_l = s_off[jl];
                }
                y_l = s_y[jl];
            }
            const int nr_l = (geo_l >> 8) & 255, ly0_l = (geo_l >> 24) & 255;
            uint64_t hits = __ballot(jl < n && ly0_l < band0 + kBand && ly0_l + nr_l > band0);
            // current run (uniform): taps [k0, kend) of the entry's rows in the
            // band; the entry's y sits in lane yl of y_l
            const C *tp = taps;
            PlaneEntry pe{};
            int k0 = 0, kend = 0, kbeg = 0, nc = 1, cell0 = 0, yl = 0;
            float inv_nc = 1.0f;
            while (hits || k0 < kend) {
                C K[kS];
                int li[kS], ys[kS];
                PlaneLoad L[kPlanes ? kS : 1];
                float sws[kPlanes ? kS : 1], sgs[kPlanes ? kS : 1];
#pragma unroll
                for (int sl = 0; sl < kS; ++sl) {
                    li[sl] = kRows * kTile;  // lanes without a tap update the spare cell by zero
                    if (k0 >= kend && hits) {  // next entry with rows in the band
                        const int l = __builtin_ctzll(hits);
                        hits &= hits - 1;
                        const int ez = __builtin_amdgcn_readlane(geo_l, l);
                        if constexpr (kPlanes) {
                            const int4 pr = make_int4(__builtin_amdgcn_readlane(prec_l.x, l),
                                                      __builtin_amdgcn_readlane(prec_l.y, l),
                                                      __builtin_amdgcn_readlane(prec_l.z, l),
                                                      __builtin_amdgcn_readlane(prec_l.w, l));
                            pe = plane_entry(pr, bcast(sw_l, l), t.table);
                        } else {
                            const int64_t off = ((int64_t)__builtin_amdgcn_readlane((int)(off_l >> 32), l) << 32) |
                                                (uint32_t)__builtin_amdgcn_readlane((int)off_l, l);
                            tp = taps + off;
                        }
                        yl = l;
                        const int nr = (ez >> 8) & 255, ly0 = (ez >> 24) & 255;
                        const int lo = ly0 > band0 ? ly0 : band0;
                        const int hi = (ly0 + nr < band0 + kBand) ? ly0 + nr : band0 + kBand;
                        nc = ez & 255;
                        kbeg = (lo - ly0) * nc;
                        kend = (hi - ly0) * nc;
                        k0 = kbeg;
                        inv_nc = recip_nc(nc);
                        cell0 = (ly0 - part * kRows) * kTile + ((ez >> 16) & 255);
                    }
                    K[sl] = zero;
                    ys[sl] = yl;
                    if constexpr (kPlanes) {
                        L[sl] = plane_zero();
                        sws[sl] = pe.sw;
                        sgs[sl] = pe.sgn;
                    }
                    if (k0 < kend) {  // uniform: this slot takes taps [k0, k0 + 64) of the run
                        const bool ok = k0 + lane < kend;
                        const int k = ok ? k0 + lane : kbeg;
                        const int row = sub_row(k, inv_nc);
                        li[sl] = ok ? sub_cell(cell0, k, row, nc) : kRows * kTile;  // else: the spare cell
                        if constexpr (kPlanes) L[sl] = plane_load(pe, row, k - (int)__umul24((unsigned)row, (unsigned)nc), t.inv_dq);
                        else K[sl] = load_tap(&tp[k]);
                        k0 += 64;
                    }
                }
#pragma unroll
                for (int sl = 0; sl < kS; ++sl) {
                    if constexpr (kPlanes) {
                        const float2 v = plane_value(L[sl], sws[sl], sgs[sl]);
                        K[sl].x = v.x;
                        K[sl].y = v.y;
                    }
                    const auto yx = bcast(y_l.x, ys[sl]), yy = bcast(y_l.y, ys[sl]);
                    const C z = tile[li[sl]];
                    C o;
                    o.x = z.x + (K[sl].x * yx + K[sl].y * yy);
                    o.y = z.y + (K[sl].x * yy - K[sl].y * yx);
                    tile[li[sl]] = o;
                }
            }
        }
    }
    const uint32_t key = t.item_key[item];
    C *dst;
    int64_t ld;
    if (t.item_sole[item]) {
        dst = tile_origin(grids, key, t);
        ld = t.G;
    } else {
        dst = (C *)t.partial + (int64_t)t.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    // the band was written by this wavefront only: no barrier needed
#pragma unroll
    for (int r = 0; r < kBand; ++r) dst[(int64_t)(band0 + r) * ld + lane] = tile[(lrow0 + r) * kTile + lane];
}

// ---- exact kernels on the band-major tap layout ------------------------------
// A unit is one band (kBR rows, 8 or 16) of one work item's 64 x 64 tile; its
// runs (the parts of the item's entries in the band) and their taps are
// contiguous in the tap array.  One wavefront serves one unit and holds the
// unit's band of the tile in LDS; the wavefronts of a block are independent
// (no block barriers), so a block only groups them for the LDS allocation.
struct RunArgs {
    const int32_t *unit_order;  // class kernels: bands by decreasing taps (block -> band)
    const int4 *clsrec;
    const int32_t *unit_cls0;
    const int4 *runrec;
    const int32_t *unit_run0;
    const int64_t *unit_tap0;
    const uint32_t *item_key;
    const uint8_t *item_sole;
    const int32_t *item_slot;
    void *partial;
    int64_t n_units;
    int tile_bits;
    int G;
};

constexpr int kRunWaves = 4;   // wavefronts (units) per block
constexpr int kClassWaves = 4; // wavefronts per band in the class kernels
constexpr int kRunChunk = 64;  // run records a grid wavefront stages in LDS at a time

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of set bits of m in lanes <= lane
__device__ __forceinline__ int bits_upto(uint64_t m, int lane) {
    const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    return below + (int)((m >> lane) & 1ull);
}

// yr[L] = yw of the visibility of run L (layout order), for k_grid_class.
template <bool kFP64>
__global__ void k_prep_runs(const typename Types<kFP64>::C *__restrict__ yw, const int4 *__restrict__ runrec,
                            int64_t R, typename Types<kFP64>::C *yr) {
    const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L < R) yr[L] = yw[runrec[L].z];
}

// y[perm[p]] = W_p (conj) sum of visibility p's run partials, in generation
// order (its entries in turn, each entry's bands in turn): deterministic.
// With lay, the partial of generation-order run g sits at dpart[lay[g]].
template <bool kFP64>
__global__ void k_degrid_reduce_runs(const typename Types<kFP64>::C *__restrict__ dpart,
                                     const int64_t *__restrict__ ent_off, const int32_t *__restrict__ run_first,
                                     const int32_t *__restrict__ lay, typename Types<kFP64>::C *vis, ApplyArgs a,
                                     int add_i) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.m) return;
    R ar = 0, ai = 0;
    const int g1 = run_first[ent_off[p + 1]];
    for (int g = run_first[ent_off[p]]; g < g1; ++g) {
        const C v = dpart[lay ? lay[g] : g];
        ar += v.x;
        ai += v.y;
    }
    const R w = (R)a.wt[p];
    C y;
    y.x = ar * w;
    y.y = (a.sflag[p] ? -ai : ai) * w;  // Eq. (8): folded visibilities are conjugated
    if (add_i) {
        C o = vis[a.perm[p]];
        o.x -= y.y;
        o.y += y.x;
        y = o;
    }
    vis[a.perm[p]] = y;
}

// GC_k^dagger (grid) on runs, no atomics: a wavefront accumulates its unit's
// band of the tile in LDS, streaming the unit's taps (one contiguous range)
// in slots of 64 consecutive taps with all lanes busy, whatever the run
// lengths.  Run records are staged 64 at a time; a slot's runs are found
// with ballots over the staged starts (a 64-bit mask of the taps that start
// a run, and each lane's count of the starts up to it).  The cells of one
// run are distinct, but two runs of a slot may share cells, so the slot's
// read-modify-writes go run by run (masked passes); a wavefront's LDS
// accesses complete in order.  The band is then stored into the grid (the
// tile's only item; an empty band is already zero there) or into the item's
// partial tile, which k_reduce_tiles sums.
template <bool kFP64, int kBR>
__global__ __launch_bounds__(64 * kRunWaves) void k_grid_runs(const typename Types<kFP64>::C *__restrict__ taps,
                                                              const typename Types<kFP64>::C *__restrict__ yw,
                                                              typename Types<kFP64>::C *grids, RunArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int kCells = kBR * kTile;
    constexpr int kNB = kTile / kBR;
    __shared__ C s_band[kRunWaves][kCells + 1];  // + a spare cell for lanes without a tap
    __shared__ int4 s_rec[kRunWaves][kRunChunk];
    __shared__ C s_y[kRunWaves][kRunChunk];
    const int wid = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * kRunWaves + wid;
    if (u >= a.n_units) return;  // uniform over the wavefront
    const int r_beg = a.unit_run0[u], r_end = a.unit_run0[u + 1];
    const int item = (int)(u / kNB), band = (int)(u % kNB);
    const bool sole = a.item_sole[item] != 0;
    if (sole && r_beg >= r_end) return;  // nothing to add to a band the zero pass cleared
    C *sb = s_band[wid];
    int4 *rec_l = s_rec[wid];
    C *y_l = s_y[wid];
    C zero;
    zero.x = 0;
    zero.y = 0;
#pragma unroll
    for (int r = 0; r < kBR; ++r) sb[r * kTile + lane] = zero;
    const C *tp = taps + a.unit_tap0[u];
    const int t_unit = (int)(a.unit_tap0[u + 1] - a.unit_tap0[u]);
    for (int c0 = r_beg; c0 < r_end; c0 += kRunChunk) {
        const int nrun = (r_end - c0 < kRunChunk) ? r_end - c0 : kRunChunk;
        wave_fence();  // the previous chunk's records are no longer read
        int st = 0x7FFFFFFF;  // start of staged run `lane` (past the chunk: never reached)
        if (lane < nrun) {
            const int4 rec = a.runrec[c0 + lane];
            rec_l[lane] = rec;
            y_l[lane] = yw[rec.z];
            st = rec.x;
        }
        wave_fence();
        const int t_beg = __builtin_amdgcn_readfirstlane(st);
        const int t_end = (c0 + nrun < r_end) ? a.runrec[c0 + nrun].x : t_unit;
        for_batches(t_beg, t_end, [&](int k0, auto ucount) {
            constexpr int U = decltype(ucount)::value;
            C K[U];
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int t = k0 + 64 * s + lane;
                K[s] = load_tap(tp + (t < t_end ? t : t_beg));
            }
#pragma unroll
            for (int s = 0; s < U; ++s) {
                const int s0 = k0 + 64 * s;
                if (s0 < t_end) {  // uniform
                    // staged run holding the slot's first tap, and the run starts inside the slot
                    const int ra = (int)__popcll(__ballot(st <= s0)) - 1;
                    uint64_t inside = __ballot(st > s0 && st <= s0 + 63);
                    const int nstarts = (int)__popcll(inside);
                    uint64_t tmask = 0;
                    while (inside) {
                        const int j = (int)__builtin_ctzll(inside);
                        inside &= inside - 1;
                        tmask |= 1ull << (__builtin_amdgcn_readlane(st, j) - s0);
                    }
                    const int rel = bits_upto(tmask, lane);
                    const int t = s0 + lane;
                    const int4 rec = rec_l[ra + rel];
                    const C y = y_l[ra + rel];
                    const int nc = (rec.y >> 16) & 255;
                    const int local = t - rec.x;
                    const int row = sub_row(local, recip_nc(nc));
                    const int cell = t < t_end ? sub_cell(rec.y & 0xFFFF, local, row, nc) : kCells;
                    const R dx = K[s].x * y.x + K[s].y * y.y;  // conj(K) y
                    const R dy = K[s].x * y.y - K[s].y * y.x;
                    for (int j = 0; j <= nstarts; ++j) {  // uniform: one pass per run of the slot
                        if (rel == j) {
                            C z = sb[cell];
                            z.x += dx;
                            z.y += dy;
                            sb[cell] = z;
                        }
                    }
                }
            }
        });
    }
    const uint32_t key = a.item_key[item];
    C *dst;
    int64_t ld;
    if (sole) {
        dst = tile_origin(grids, key, a.tile_bits, a.G);
        ld = a.G;
    } else {
        dst = (C *)a.partial + (int64_t)a.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    dst += (int64_t)band * kBR * ld;
    wave_fence();
#pragma unroll
    for (int r = 0; r < kBR; ++r) dst[(int64_t)r * ld + lane] = sb[r * kTile + lane];
}

// ---- exact kernels on run classes (contiguous-runs layout) ---------------
// Neighbouring runs of one shape (same width, rows and first cell: the same
// band cells) form a class; visibilities are dense in uv, so a class holds
// tens of runs.  A wavefront serves a unit class by class with one lane per
// tap of the shape: grid accumulates conj(K) y of the class's runs in
// registers and updates the band once per class (no atomics, no conflicts);
// degrid multiplies each run's taps by the band values it holds in registers
// and sums them across the lanes.  Shapes of at most 64 taps use slices of W
// lanes (W the next power of two), 64 / W runs at a time; longer shapes use
// all 64 lanes per chunk of 64 taps.
// runs per slice (short shapes) and runs (long shapes) whose loads are issued together
constexpr int kDegridUnroll = 4, kDegridLongUnroll = 8;
constexpr int kGridUnroll = 4, kGridLongUnroll = 8;

// Sum over aligned blocks of W lanes with DPP moves; the block's sum ends in
// its last lane.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add_src(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xF, false));
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_add_src(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, kRowMask, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int W, typename R>
__device__ __forceinline__ R block_sum_last(R v) {
    if constexpr (W >= 2) v += dpp_add_src<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
    if constexpr (W >= 4) v += dpp_add_src<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
    if constexpr (W >= 8) v += dpp_add_src<0x141, 0xF>(v);  // row_half_mirror
    if constexpr (W >= 16) v += dpp_add_src<0x140, 0xF>(v); // row_mirror
    if constexpr (W >= 32) v += dpp_add_src<0x142, 0xA>(v); // row_bcast:15 into rows 1, 3
    if constexpr (W >= 64) v += dpp_add_src<0x143, 0xC>(v); // row_bcast:31 into rows 2, 3
    return v;
}

__device__ __forceinline__ int pow2_at_least(int x) {
    int w = 1;
    while (w < x) w <<= 1;
    return w;
}

// Degrid of one class with slices of W lanes (shape of L <= W taps).
// Run partials go to dpart in layout order (dpart[run0 + i]).
template <bool kFP64, int W>
__device__ __forceinline__ void degrid_class_small(const typename Types<kFP64>::C *__restrict__ tp,
                                                   typename Types<kFP64>::C z, int L, int m,
                                                   typename Types<kFP64>::C *dpart, int lane) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int P = 64 / W;
    const int sl = lane / W, kk = lane % W;
    const bool act = kk < L;
    for (int i0 = 0; i0 < m; i0 += P * kDegridUnroll) {
        C K[kDegridUnroll];
#pragma unroll
        for (int j = 0; j < kDegridUnroll; ++j) {
            const int i = i0 + j * P + sl;
            K[j].x = 0;
            K[j].y = 0;
            if (act && i < m) K[j] = load_tap(tp + (uint32_t)(i * L + kk));
        }
#pragma unroll
        for (int j = 0; j < kDegridUnroll; ++j) {
            R pr = K[j].x * z.x - K[j].y * z.y;
            R pi = K[j].x * z.y + K[j].y * z.x;
            pr = block_sum_last<W>(pr);
            pi = block_sum_last<W>(pi);
            const int i = i0 + j * P + sl;
            if (kk == W - 1 && i < m) {
                C o;
                o.x = pr;
                o.y = pi;
                dpart[i] = o;
            }
        }
    }
}

// A block serves one band: its kClassWaves wavefronts stage the band together
// and then take every kClassWaves-th class each (classes are independent in
// degrid), so that a large band is not left to one wavefront at the end of
// the launch (a wavefront streams at a small fraction of the chip's rate).
// Blocks take the bands in decreasing order of taps, so that the launch ends
// on small ones.
template <bool kFP64, int kBR>
__global__ __launch_bounds__(64 * kClassWaves) void k_degrid_class(const typename Types<kFP64>::C *__restrict__ taps,
                                                                 const typename Types<kFP64>::C *__restrict__ grids,
                                                                 typename Types<kFP64>::C *dpart, RunArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ C sb[kBR * kTile];
    const int wid = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = a.unit_order[blockIdx.x];
    const int c_first = a.unit_cls0[u], c_end = a.unit_cls0[u + 1];
    if (c_first >= c_end) return;  // uniform over the block
    constexpr int kNB = kTile / kBR;
    const int item = (int)(u / kNB), band = (int)(u % kNB);
    {
        const C *src = tile_origin(grids, a.item_key[item], a.tile_bits, a.G) + (int64_t)band * kBR * a.G;
        for (int r = wid; r < kBR; r += kClassWaves) sb[r * kTile + lane] = src[(int64_t)r * a.G + lane];
    }
    __syncthreads();
    const C *tu = taps + a.unit_tap0[u];
    for (int c = c_first + wid; c < c_end; c += kClassWaves) {
        const int4 cr = a.clsrec[c];
        const int nc = (cr.w >> 16) & 255, nrows = (cr.w >> 24) & 255, cell0 = cr.w & 0xFFFF;
        const int L = nc * nrows, run0 = cr.y, m = cr.z;
        const C *tp = tu + cr.x;
        if (L <= 64) {
            const int W = pow2_at_least(L);
            const int kk = lane % W;
            C z;
            z.x = 0;
            z.y = 0;
            if (kk < L) z = sb[cell0 + (kk / nc) * kTile + kk % nc];
            C *dp = dpart + run0;
            switch (W) {
            case 1: degrid_class_small<kFP64, 1>(tp, z, L, m, dp, lane); break;
            case 2: degrid_class_small<kFP64, 2>(tp, z, L, m, dp, lane); break;
            case 4: degrid_class_small<kFP64, 4>(tp, z, L, m, dp, lane); break;
            case 8: degrid_class_small<kFP64, 8>(tp, z, L, m, dp, lane); break;
            case 16: degrid_class_small<kFP64, 16>(tp, z, L, m, dp, lane); break;
            case 32: degrid_class_small<kFP64, 32>(tp, z, L, m, dp, lane); break;
            default: degrid_class_small<kFP64, 64>(tp, z, L, m, dp, lane); break;
            }
        } else {
            // long shapes: kDegridLongUnroll runs at a time, 64 taps per step, band values from LDS
            for (int i0 = 0; i0 < m; i0 += kDegridLongUnroll) {
                R pr[kDegridLongUnroll], pi[kDegridLongUnroll];
#pragma unroll
                for (int j = 0; j < kDegridLongUnroll; ++j) pr[j] = pi[j] = 0;
                for (int k0 = 0; k0 < L; k0 += 64) {
                    const int k = k0 + lane;
                    C K[kDegridLongUnroll];
#pragma unroll
                    for (int j = 0; j < kDegridLongUnroll; ++j) {
                        K[j].x = 0;
                        K[j].y = 0;
                        if (k < L && i0 + j < m) K[j] = load_tap(tp + (uint32_t)((i0 + j) * L + k));
                    }
                    C z;
                    z.x = 0;
                    z.y = 0;
                    if (k < L) z = sb[cell0 + (k / nc) * kTile + k % nc];
#pragma unroll
                    for (int j = 0; j < kDegridLongUnroll; ++j) {
                        pr[j] += K[j].x * z.x - K[j].y * z.y;
                        pi[j] += K[j].x * z.y + K[j].y * z.x;
                    }
                }
#pragma unroll
                for (int j = 0; j < kDegridLongUnroll; ++j) {
                    const R sr = block_sum_last<64>(pr[j]);
                    const R si = block_sum_last<64>(pi[j]);
                    if (lane == 63 && i0 + j < m) {
                        C o;
                        o.x = sr;
                        o.y = si;
                        dpart[run0 + i0 + j] = o;
                    }
                }
            }
        }
    }
}

// Grid of one class with slices of W lanes: returns the lane's sum over the
// class's runs of conj(K) y for its tap (slices combined).
// yr: the class's runs' weighted visibilities, in layout order.
template <bool kFP64, int W>
__device__ __forceinline__ typename Types<kFP64>::C grid_class_small(const typename Types<kFP64>::C *__restrict__ tp,
                                                                     const typename Types<kFP64>::C *__restrict__ yr,
                                                                     int L, int m, int lane) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int P = 64 / W;
    const int sl = lane / W, kk = lane % W;
    const bool act = kk < L;
    R ar = 0, ai = 0;
    for (int i0 = 0; i0 < m; i0 += P * kGridUnroll) {
        C K[kGridUnroll], y[kGridUnroll];
#pragma unroll
        for (int j = 0; j < kGridUnroll; ++j) {
            const int i = i0 + j * P + sl;
            K[j].x = K[j].y = y[j].x = y[j].y = 0;
            if (i < m) y[j] = yr[i];
            if (act && i < m) K[j] = load_tap(tp + (uint32_t)(i * L + kk));
        }
#pragma unroll
        for (int j = 0; j < kGridUnroll; ++j) {
            ar += K[j].x * y[j].x + K[j].y * y[j].y;  // conj(K) y
            ai += K[j].x * y[j].y - K[j].y * y[j].x;
        }
    }
#pragma unroll
    for (int o = W; o < 64; o <<= 1) {  // slices hold other runs of the same taps
        ar += __shfl_xor(ar, o, 64);
        ai += __shfl_xor(ai, o, 64);
    }
    C out;
    out.x = ar;
    out.y = ai;
    return out;
}

// Grid on run classes: a block serves one band; each of its wavefronts takes
// every kClassWaves-th class and accumulates into its own copy of the band in
// LDS (a class's cells are distinct; classes go in program order), then the
// block sums the copies in wavefront order (deterministic) and stores the band.
template <bool kFP64, int kBR>
__global__ __launch_bounds__(64 * kClassWaves) void k_grid_class(const typename Types<kFP64>::C *__restrict__ taps,
                                                                 const typename Types<kFP64>::C *__restrict__ yr,
                                                                 typename Types<kFP64>::C *grids, RunArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ C s_band[kClassWaves][kBR * kTile];
    const int wid = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = a.unit_order[blockIdx.x];
    const int c_first = a.unit_cls0[u], c_end = a.unit_cls0[u + 1];
    constexpr int kNB = kTile / kBR;
    const int item = (int)(u / kNB), band = (int)(u % kNB);
    const bool sole = a.item_sole[item] != 0;
    if (sole && c_first >= c_end) return;  // uniform over the block: the zero pass cleared the band
    C *sb = s_band[wid];
    C zero;
    zero.x = 0;
    zero.y = 0;
#pragma unroll
    for (int r = 0; r < kBR; ++r) sb[r * kTile + lane] = zero;
    wave_fence();
    const C *tu = taps + a.unit_tap0[u];
    for (int c = c_first + wid; c < c_end; c += kClassWaves) {
        const int4 cr = a.clsrec[c];
        const int nc = (cr.w >> 16) & 255, nrows = (cr.w >> 24) & 255, cell0 = cr.w & 0xFFFF;
        const int L = nc * nrows, run0 = cr.y, m = cr.z;
        const C *tp = tu + cr.x;
        if (L <= 64) {
            const int W = pow2_at_least(L);
            C acc;
            const C *yc = yr + run0;
            switch (W) {
            case 1: acc = grid_class_small<kFP64, 1>(tp, yc, L, m, lane); break;
            case 2: acc = grid_class_small<kFP64, 2>(tp, yc, L, m, lane); break;
            case 4: acc = grid_class_small<kFP64, 4>(tp, yc, L, m, lane); break;
            case 8: acc = grid_class_small<kFP64, 8>(tp, yc, L, m, lane); break;
            case 16: acc = grid_class_small<kFP64, 16>(tp, yc, L, m, lane); break;
            case 32: acc = grid_class_small<kFP64, 32>(tp, yc, L, m, lane); break;
            default: acc = grid_class_small<kFP64, 64>(tp, yc, L, m, lane); break;
            }
            if (lane < L) {  // slice 0 holds the combined sums; the class's cells are distinct
                const int cell = cell0 + (lane / nc) * kTile + lane % nc;
                C v = sb[cell];
                v.x += acc.x;
                v.y += acc.y;
                sb[cell] = v;
            }
        } else {
            // long shapes (> 64 taps): the class's taps in order, 64 consecutive taps per
            // step, so the 64 lanes of a step hold distinct taps of at most two runs, on
            // distinct cells: a plain read-modify-write per step
            const float inv_nc = recip_nc(nc);
            const int total = m * L;
            int i = 0, k = lane;  // run and tap of the lane's current tap (L > 64: lane < L)
            for (int t0 = 0; t0 < total; t0 += 64 * kGridLongUnroll) {
                C K[kGridLongUnroll], y[kGridLongUnroll];
                int cell[kGridLongUnroll];
#pragma unroll
                for (int j = 0; j < kGridLongUnroll; ++j) {
                    const bool on = t0 + 64 * j + lane < total;
                    K[j].x = K[j].y = y[j].x = y[j].y = 0;
                    cell[j] = 0;
                    if (on) {
                        K[j] = load_tap(tp + t0 + 64 * j + lane);
                        y[j] = yr[run0 + i];
                        const int row = sub_row(k, inv_nc);
                        cell[j] = sub_cell(cell0, k, row, nc);
                    }
                    k += 64;
                    if (k >= L) {  // one wrap at most: L > 64
                        k -= L;
                        ++i;
                    }
                }
#pragma unroll
                for (int j = 0; j < kGridLongUnroll; ++j) {
                    if (t0 + 64 * j + lane < total) {
                        C v = sb[cell[j]];
                        v.x += K[j].x * y[j].x + K[j].y * y[j].y;  // conj(K) y
                        v.y += K[j].x * y[j].y - K[j].y * y[j].x;
                        sb[cell[j]] = v;
                    }
                }
            }
        }
    }
    const uint32_t key = a.item_key[item];
    C *dst;
    int64_t ld;
    if (sole) {
        dst = tile_origin(grids, key, a.tile_bits, a.G);
        ld = a.G;
    } else {
        dst = (C *)a.partial + (int64_t)a.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    dst += (int64_t)band * kBR * ld;
    __syncthreads();
    for (int r = wid; r < kBR; r += kClassWaves) {
        C v = s_band[0][r * kTile + lane];
#pragma unroll
        for (int w = 1; w < kClassWaves; ++w) {
            const C t = s_band[w][r * kTile + lane];
            v.x += t.x;
            v.y += t.y;
        }
        dst[(int64_t)r * ld + lane] = v;
    }
}

// ---- exact kernels on the interleaved tap layout -------------------------
// Short runs (many w-stacks, supports of a few cells): one wavefront per unit
// as above, but lane i serves run i of each group of 64 of the unit's runs
// (longest first).  Step k of a group reads tap k of every run at least k + 1
// long, a contiguous range of the tap array, so every load instruction is
// coalesced and no lane ever looks for the run a tap belongs to.  A lane
// walks its run's cells row by row within the band.  kLaneSteps steps' loads
// are issued before their taps are used.
constexpr int kLaneSteps = 8;

// GC_k, W_k (degrid): each lane's run partial goes to dpart at the run's
// generation index; k_degrid_reduce_runs sums them per visibility.
template <bool kFP64, int kBR>
__global__ __launch_bounds__(64 * kRunWaves) void k_degrid_lanes(const typename Types<kFP64>::C *__restrict__ taps,
                                                                 const typename Types<kFP64>::C *__restrict__ grids,
                                                                 typename Types<kFP64>::C *dpart, RunArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ C s_band[kRunWaves][kBR * kTile];
    const int wid = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * kRunWaves + wid;
    if (u >= a.n_units) return;  // uniform over the wavefront
    const int r_beg = a.unit_run0[u], r_end = a.unit_run0[u + 1];
    if (r_beg >= r_end) return;
    constexpr int kNB = kTile / kBR;
    const int item = (int)(u / kNB), band = (int)(u % kNB);
    C *sb = s_band[wid];
    {
        const C *src = tile_origin(grids, a.item_key[item], a.tile_bits, a.G) + (int64_t)band * kBR * a.G;
#pragma unroll
        for (int r = 0; r < kBR; ++r) sb[r * kTile + lane] = src[(int64_t)r * a.G + lane];
    }
    wave_fence();
    const C *tp = taps + a.unit_tap0[u];
    for (int g0 = r_beg; g0 < r_end; g0 += 64) {
        const int4 rec = a.runrec[g0 + lane];
        const int nc = (rec.y >> 16) & 255;
        const int len = nc * ((rec.y >> 24) & 255);
        const int lmax = __builtin_amdgcn_readfirstlane(len);  // lane 0 holds the longest run
        const C *gp = tp + __builtin_amdgcn_readfirstlane(rec.x);
        int cell = rec.y & 0xFFFF, col = 0;
        int S = 0;  // taps of the group stored before the current step
        R ar = 0, ai = 0;
        for (int k0 = 0; k0 < lmax; k0 += kLaneSteps) {
            C K[kLaneSteps];
#pragma unroll
            for (int j = 0; j < kLaneSteps; ++j) {
                const bool on = k0 + j < len;
                K[j].x = 0;
                K[j].y = 0;
                if (on) K[j] = load_tap(gp + S + lane);
                S += (int)__popcll(__ballot(on));
            }
#pragma unroll
            for (int j = 0; j < kLaneSteps; ++j) {
                const C z = sb[k0 + j < len ? cell : 0];  // K = 0 past the run's end
                ar += K[j].x * z.x - K[j].y * z.y;
                ai += K[j].x * z.y + K[j].y * z.x;
                ++col;
                ++cell;
                if (col == nc) {
                    col = 0;
                    cell += kTile - nc;
                }
            }
        }
        if (rec.w >= 0) {
            C o;
            o.x = ar;
            o.y = ai;
            dpart[rec.w] = o;
        }
    }
}

// GC_k^dagger (grid): each lane adds conj(K) y of its run into the band in
// LDS with LDS atomic adds (runs of a step may share cells); the band is then
// stored as in k_grid_runs.
template <bool kFP64, int kBR>
__global__ __launch_bounds__(64 * kRunWaves) void k_grid_lanes(const typename Types<kFP64>::C *__restrict__ taps,
                                                               const typename Types<kFP64>::C *__restrict__ yw,
                                                               typename Types<kFP64>::C *grids, RunArgs a) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    __shared__ C s_band[kRunWaves][kBR * kTile];
    const int wid = wave_index();
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * kRunWaves + wid;
    if (u >= a.n_units) return;  // uniform over the wavefront
    const int r_beg = a.unit_run0[u], r_end = a.unit_run0[u + 1];
    constexpr int kNB = kTile / kBR;
    const int item = (int)(u / kNB), band = (int)(u % kNB);
    const bool sole = a.item_sole[item] != 0;
    if (sole && r_beg >= r_end) return;  // nothing to add to a band the zero pass cleared
    C *sb = s_band[wid];
    C zero;
    zero.x = 0;
    zero.y = 0;
#pragma unroll
    for (int r = 0; r < kBR; ++r) sb[r * kTile + lane] = zero;
    wave_fence();
    const C *tp = taps + a.unit_tap0[u];
    for (int g0 = r_beg; g0 < r_end; g0 += 64) {
        const int4 rec = a.runrec[g0 + lane];
        const int nc = (rec.y >> 16) & 255;
        const int len = nc * ((rec.y >> 24) & 255);
        const int lmax = __builtin_amdgcn_readfirstlane(len);
        const C *gp = tp + __builtin_amdgcn_readfirstlane(rec.x);
        const C y = rec.w >= 0 ? yw[rec.z] : zero;
        int cell = rec.y & 0xFFFF, col = 0;
        int S = 0;
        for (int k0 = 0; k0 < lmax; k0 += kLaneSteps) {
            C K[kLaneSteps];
#pragma unroll
            for (int j = 0; j < kLaneSteps; ++j) {
                const bool on = k0 + j < len;
                K[j].x = 0;
                K[j].y = 0;
                if (on) K[j] = load_tap(gp + S + lane);
                S += (int)__popcll(__ballot(on));
            }
#pragma unroll
            for (int j = 0; j < kLaneSteps; ++j) {
                if (k0 + j < len) {
                    atomicAdd(&sb[cell].x, K[j].x * y.x + K[j].y * y.y);  // conj(K) y
                    atomicAdd(&sb[cell].y, K[j].x * y.y - K[j].y * y.x);
                }
                ++col;
                ++cell;
                if (col == nc) {
                    col = 0;
                    cell += kTile - nc;
                }
            }
        }
    }
    const uint32_t key = a.item_key[item];
    C *dst;
    int64_t ld;
    if (sole) {
        dst = tile_origin(grids, key, a.tile_bits, a.G);
        ld = a.G;
    } else {
        dst = (C *)a.partial + (int64_t)a.item_slot[item] * kTile * kTile;
        ld = kTile;
    }
    dst += (int64_t)band * kBR * ld;
    wave_fence();
#pragma unroll
    for (int r = 0; r < kBR; ++r) dst[(int64_t)r * ld + lane] = sb[r * kTile + lane];
}

// Sum the partial tiles of each tile shared by several items, in the order of
// the tile's items (deterministic), and store the result in the grid.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_reduce_tiles(const int32_t *__restrict__ mt_first,
                                                      typename Types<kFP64>::C *grids, TileArgs t) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    // positions a .. b - 1 of t.itile are the tile's items; their slots are consecutive
    const int a = mt_first[blockIdx.x];
    const uint32_t key = t.item_key[t.itile[a]];
    int b = a + 1;
    while (b < t.n_items && t.item_key[t.itile[b]] == key) ++b;
    const int slot0 = t.item_slot[t.itile[a]];
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
    a.iperm = pl.iperm;
    a.wt_in = pl.wt_in;
    a.flag = pl.flag;
    a.tap_off = pl.tap_off;
    a.m = pl.m;
    a.g = c->g;
    return a;
}

template <typename C>
hipfftResult fft_pass(hipfftHandle plan, C *data, int dir, hipStream_t s) {
    hipfftResult r = hipfftSetStream(plan, s);
    if (r != HIPFFT_SUCCESS) return r;
    if constexpr (sizeof(C) == 16) {
        return hipfftExecZ2Z(plan, (hipfftDoubleComplex *)data, (hipfftDoubleComplex *)data, dir);
    } else {
        return hipfftExecC2C(plan, (hipfftComplex *)data, (hipfftComplex *)data, dir);
    }
}

// The U pass over the used rows of every stack: rows [0, rows_lo) of stack
// 0, then each stack's top band with the next stack's bottom band (adjacent
// in memory), then the last stack's top band.
template <typename C>
hipError_t u_pass(wsp_ctx *c, C *grids, int dir, hipStream_t s) {
    const Geom &g = c->g;
    if (g.rows_lo >= g.G) return fft_pass(c->fft_u, grids, dir, s) == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown;
    const int64_t GG = (int64_t)g.G * g.G;
    if (c->fft_ulo_made && fft_pass(c->fft_ulo, grids, dir, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
    for (int k = 0; k + 1 < g.n_stacks; ++k) {
        C *band = grids + k * GG + (int64_t)(g.G - g.rows_hi) * g.G;
        if (fft_pass(c->fft_ujoin, band, dir, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
    }
    if (c->fft_uhi_made) {
        C *band = grids + (int64_t)(g.n_stacks - 1) * GG + (int64_t)(g.G - g.rows_hi) * g.G;
        if (fft_pass(c->fft_uhi, band, dir, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
    }
    return hipSuccess;
}

// F (forward, from H to the grids) or F^dagger (backward, from the grids to H),
// both unnormalised.
template <typename C>
hipError_t fft_exec(wsp_ctx *c, bool forward, hipStream_t s) {
    const Geom &g = c->g;
    C *grids = (C *)c->grids, *half = (C *)c->scratch_half;
    const dim3 tgrid((unsigned)(g.G / kT), (unsigned)((g.n + kT - 1) / kT), (unsigned)g.n_stacks);
    if (forward) {
        if (fft_pass(c->fft_v, half, HIPFFT_FORWARD, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
        hipLaunchKernelGGL(k_transpose_pad<C>, dim3(g.G / kT, g.G / kT, g.n_stacks), dim3(256), 0, s,
                           (const C *)half, grids, g);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = u_pass<C>(c, grids, HIPFFT_FORWARD, s);
        if (e != hipSuccess) return e;
    } else {
        hipError_t e = u_pass<C>(c, grids, HIPFFT_BACKWARD, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_transpose_crop<C>, tgrid, dim3(256), 0, s, (const C *)grids, half, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (fft_pass(c->fft_v, half, HIPFFT_BACKWARD, s) != HIPFFT_SUCCESS) return hipErrorUnknown;
    }
    return hipSuccess;
}

// Grid kernel choice for the contiguous-runs layout: when most taps are in
// shapes longer than 64 taps (large supports), k_grid_runs streams each band's
// taps in 64-tap steps with fewer registers and outruns the class kernel
// (measured on 1024^2 single-stack and 4096^2 16-stack MWA-like workloads);
// otherwise k_grid_class accumulates each class in registers.
static bool grid_on_runs(const Plan &pl) { return 2 * pl.long_taps > pl.total_taps; }

RunArgs run_args(const wsp_ctx *c) {
    const Plan &pl = c->plan;
    RunArgs r{};
    r.unit_order = pl.unit_order;
    r.clsrec = pl.clsrec;
    r.unit_cls0 = pl.unit_cls0;
    r.runrec = pl.runrec;
    r.unit_run0 = pl.unit_run0;
    r.unit_tap0 = pl.unit_tap0;
    r.item_key = pl.item_key;
    r.item_sole = pl.item_sole;
    r.item_slot = pl.item_slot;
    r.partial = c->scratch_part;
    r.n_units = (int64_t)pl.n_items * pl.tile_bands;
    r.tile_bits = pl.tile_bits;
    r.G = c->g.G;
    return r;
}

void set_plane_args(const wsp_ctx *c, TileArgs *ta) {
    ta->itile = c->plan.itile;
    if (!c->g.planes) return;
    ta->prec = c->plan.prec;
    ta->ptw = c->plan.ptw;
    ta->table = (const float4 *)c->taps;
    ta->inv_dq = (float)c->g.plane_inv_dq;
}

// w-plane mode test hook: the J_p x J_p taps of sorted visibility sidx,
// row-major, interpolated exactly as the tile kernels do (the sub-block is
// the whole support).
__global__ void k_plane_vis_taps(const double *__restrict__ ux, const double *__restrict__ vx,
                                 const double *__restrict__ weff, const int32_t *__restrict__ jp,
                                 const int64_t *__restrict__ plane_off, int n_pairs, double inv_dw,
                                 const float4 *__restrict__ table, float inv_dq, int64_t sidx,
                                 float2 *out) {
    const int J = jp[sidx];
    int4 rec;
    float sw;
    plane_record(weff[sidx], ux[sidx], vx[sidx], plane_off, n_pairs, inv_dw, &rec, &sw);
    const PlaneEntry pe = plane_entry(rec, sw, table);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < J * J; t += gridDim.x * blockDim.x) {
        const int row = t / J, col = t - row * J;
        out[t] = plane_value(plane_load(pe, row, col, inv_dq), pe.sw, pe.sgn);
    }
}

// Test hook: the J_p x J_p taps of sorted visibility sidx, row-major, read
// from their positions in the band-major layout.
template <typename C>
__global__ void k_vis_taps(const C *__restrict__ taps, TapLayout lay, const int32_t *__restrict__ jp,
                           const int32_t *__restrict__ u0w, const int32_t *__restrict__ v0w, int64_t sidx, C *out) {
    const int J = jp[sidx];
    const int uw = u0w[sidx], vw = v0w[sidx];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < J * J; t += gridDim.x * blockDim.x) {
        const int row = t / J, col = t - row * J;
        out[t] = taps[tap_position(lay, (int)sidx, row, col, J, uw, vw)];
    }
}

template <bool kFP64>
hipError_t degrid_t(wsp_ctx *c, const void *image, void *vis, const double *d_centres,
                    hipStream_t s, int add_i) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const Geom &g = c->g;
    hipEvent_t ev = stage_begin(c, s);
    hipError_t e;
    if (c->fft_lds) {
        e = fft_lds_image_in<kFP64>(g, image, c->scratch_half, s);
        stage_end(c, kStTaperPad, ev, s);
        if (e != hipSuccess) return e;
        ev = stage_begin(c, s);
        e = fft_lds_forward<kFP64>(g, c->grids, c->scratch_half, c->fft_tw, c->fft_tile_bits, d_centres, 0,
                                   g.n_stacks, s);
        stage_end(c, kStFftForward, ev, s);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_taper_half<kFP64>, dim3(g.G / kT, (g.n + kT - 1) / kT), dim3(256), 0, s,
                           (const R *)image, (C *)c->scratch_half, d_centres, g);
        stage_end(c, kStTaperPad, ev, s);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ev = stage_begin(c, s);
        e = fft_exec<C>(c, true, s);
        stage_end(c, kStFftForward, ev, s);
        if (e != hipSuccess) return e;
    }
    ApplyArgs a = make_args(c);
    const Plan &pl = c->plan;
    const C *tp = (const C *)c->taps;
    const C *gr = (const C *)c->grids;
    C *dp = (C *)c->scratch_dpart;
    ev = stage_begin(c, s);
    if (!g.planes) {
        const RunArgs ra = run_args(c);
        if (ra.n_units > 0) {
            const dim3 gd(blocks(ra.n_units, kRunWaves)), bd(64 * kRunWaves);
            if (pl.interleaved) {
                if (pl.tile_band_rows == 16) hipLaunchKernelGGL((k_degrid_lanes<kFP64, 16>), gd, bd, 0, s, tp, gr, dp, ra);
                else hipLaunchKernelGGL((k_degrid_lanes<kFP64, 8>), gd, bd, 0, s, tp, gr, dp, ra);
            } else {
                const dim3 gs((unsigned)ra.n_units), bs(64 * kClassWaves);  // one block per band
                if (pl.tile_band_rows == 16) hipLaunchKernelGGL((k_degrid_class<kFP64, 16>), gs, bs, 0, s, tp, gr, dp, ra);
                else hipLaunchKernelGGL((k_degrid_class<kFP64, 8>), gs, bs, 0, s, tp, gr, dp, ra);
            }
        }
        // class kernels write run partials in layout order
        const int32_t *lay = pl.interleaved ? nullptr : pl.run_lay;
        hipLaunchKernelGGL(k_degrid_reduce_runs<kFP64>, dim3(blocks(a.m, 256)), dim3(256), 0, s, (const C *)dp,
                           pl.ent_off, pl.run_first, lay, (C *)vis, a, add_i);
        stage_end(c, kStDegrid, ev, s);
        return hipGetLastError();
    }
    TileArgs ta{pl.wrec,      pl.ent_sorted,   pl.item_start, pl.item_key, pl.item_sole,
                pl.item_slot, c->scratch_part, pl.n_items,    pl.tile_bits, g.G};
    set_plane_args(c, &ta);
    if constexpr (!kFP64) {  // w-plane kernels (FP32 path only)
        if (pl.n_items > 0) {
            const unsigned nb = (unsigned)(8 * ((pl.n_items + 7) / 8));
            // entries of a few tens of taps (many w-stacks) go four to a wavefront
            const bool small = pl.total_taps < kSmallEntryTaps * pl.n_entries;
            if (small) hipLaunchKernelGGL((k_degrid_small<false, true>), dim3(nb), dim3(kThreads), 0, s, tp, gr, dp, ta);
            else hipLaunchKernelGGL((k_degrid_tiles<false, true>), dim3(nb), dim3(kThreads), 0, s, tp, gr, dp, ta);
        }
    }
    hipLaunchKernelGGL(k_degrid_reduce<kFP64>, dim3(blocks(a.m, 256)), dim3(256), 0, s,
                       (const C *)c->scratch_dpart, pl.ent_off, (C *)vis, a, add_i);
    stage_end(c, kStDegrid, ev, s);
    return hipGetLastError();
}

template <bool kFP64>
hipError_t grid_t(wsp_ctx *c, const void *vis, void *image, const double *d_centres,
                  hipStream_t s, int rot) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    const Geom &g = c->g;
    const int64_t ncell = (int64_t)(g.rows_lo + g.rows_hi) * g.G * g.n_stacks;
    hipEvent_t ev = stage_begin(c, s);
    if (c->fft_lds)  // F^dagger reads only the used tiles
        fft_lds_zero_tiles<kFP64>(g, c->grids, c->fft_tile_list, c->n_fft_tiles, c->plan.tile_bits, s);
    else
        hipLaunchKernelGGL(k_zero_rows<C>, dim3(blocks(ncell, 256)), dim3(256), 0, s, (C *)c->grids, g);
    stage_end(c, kStZero, ev, s);
    ApplyArgs a = make_args(c);
    const Plan &pl = c->plan;
    TileArgs ta{pl.wrec,      pl.ent_sorted,   pl.item_start, pl.item_key, pl.item_sole,
                pl.item_slot, c->scratch_part, pl.n_items,    pl.tile_bits, g.G};
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_prep_vis<kFP64>, dim3(blocks(a.m, 256)), dim3(256), 0, s, (const C *)vis,
                       (C *)c->scratch_yw, a, rot);
    set_plane_args(c, &ta);
    const C *tp = (const C *)c->taps;
    const C *yw = (const C *)c->scratch_yw;
    C *gr = (C *)c->grids;
    if (!g.planes) {
        const RunArgs ra = run_args(c);
        const dim3 gd(blocks(ra.n_units, kRunWaves)), bd(64 * kRunWaves);
        if (ra.n_units > 0 && pl.interleaved) {
            if (pl.tile_band_rows == 16) hipLaunchKernelGGL((k_grid_lanes<kFP64, 16>), gd, bd, 0, s, tp, yw, gr, ra);
            else hipLaunchKernelGGL((k_grid_lanes<kFP64, 8>), gd, bd, 0, s, tp, yw, gr, ra);
        } else if (ra.n_units > 0 && grid_on_runs(pl)) {
            if (pl.tile_band_rows == 16) hipLaunchKernelGGL((k_grid_runs<kFP64, 16>), gd, bd, 0, s, tp, yw, gr, ra);
            else hipLaunchKernelGGL((k_grid_runs<kFP64, 8>), gd, bd, 0, s, tp, yw, gr, ra);
        } else if (ra.n_units > 0) {
            // each run's weighted visibility in layout order (the partials' space is free here)
            C *yr = (C *)c->scratch_dpart;
            hipLaunchKernelGGL(k_prep_runs<kFP64>, dim3(blocks(pl.n_runs, 256)), dim3(256), 0, s, yw, pl.runrec,
                               pl.n_runs, yr);
            const dim3 gs((unsigned)ra.n_units), bs(64 * kClassWaves);  // one block per band
            if (pl.tile_band_rows == 16) hipLaunchKernelGGL((k_grid_class<kFP64, 16>), gs, bs, 0, s, tp, yr, gr, ra);
            else hipLaunchKernelGGL((k_grid_class<kFP64, 8>), gs, bs, 0, s, tp, yr, gr, ra);
        }
    } else if constexpr (!kFP64) {  // w-plane kernels (FP32 path only)
        if (pl.n_items > 0) {
            const unsigned nb = (unsigned)(8 * ((pl.n_items + 7) / 8));
            const bool small = pl.total_taps < kSmallEntryTaps * pl.n_entries;
            const dim3 gs(kGridSplitSmall * nb), bs(kThreads / kGridSplitSmall);
            const dim3 gt(kGridSplit * nb), bt(kThreads / kGridSplit);
            if (small) hipLaunchKernelGGL((k_grid_small<false, kGridSplitSmall, true>), gs, bs, 0, s, tp, yw, gr, ta);
            else hipLaunchKernelGGL((k_grid_tiles<false, kGridSplit, true>), gt, bt, 0, s, tp, yw, gr, ta);
        }
    }
    if (pl.n_mtiles > 0) {
        hipLaunchKernelGGL(k_reduce_tiles<kFP64>, dim3(pl.n_mtiles), dim3(256), 0, s, pl.mt_first,
                           (C *)c->grids, ta);
    }
    stage_end(c, kStGrid, ev, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ev = stage_begin(c, s);
    if (c->fft_lds) {
        e = fft_lds_inverse<kFP64>(g, c->grids, c->scratch_half, c->fft_tw, c->fft_tile_bits, 0, g.n_stacks, s);
        stage_end(c, kStFftInverse, ev, s);
        if (e != hipSuccess) return e;
        ev = stage_begin(c, s);
        e = fft_lds_image_out<kFP64>(g, image, c->scratch_half, c->fft_tw, d_centres, s);
        stage_end(c, kStCropUntaper, ev, s);
        return e;
    }
    e = fft_exec<C>(c, false, s);
    stage_end(c, kStFftInverse, ev, s);
    if (e != hipSuccess) return e;
    ev = stage_begin(c, s);
    hipLaunchKernelGGL(k_crop_half<kFP64>, dim3((g.n + kT - 1) / kT, (g.n + kT - 1) / kT), dim3(256),
                       0, s, (const C *)c->scratch_half, (R *)image, d_centres, g);
    stage_end(c, kStCropUntaper, ev, s);
    return hipGetLastError();
}

}  // namespace

hipError_t run_degrid(wsp_ctx *c, const void *image, void *vis, hipStream_t s, int add_i) {
    if (c->p.precision == WSP_FP64) return degrid_t<true>(c, image, vis, c->plan_centres, s, add_i);
    return degrid_t<false>(c, image, vis, c->plan_centres, s, add_i);
}

hipError_t run_grid(wsp_ctx *c, const void *vis, void *image, hipStream_t s, int rot) {
    if (c->p.precision == WSP_FP64) return grid_t<true>(c, vis, image, c->plan_centres, s, rot);
    return grid_t<false>(c, vis, image, c->plan_centres, s, rot);
}

hipError_t run_exact_taps(wsp_ctx *c, int64_t sidx, void *out_dev, hipStream_t s) {
    const Plan &pl = c->plan;
    const TapLayout lay = tap_layout(pl);
    if (c->p.precision == WSP_FP64)
        hipLaunchKernelGGL(k_vis_taps<double2>, dim3(64), dim3(256), 0, s, (const double2 *)c->taps, lay, pl.jp,
                           pl.u0w, pl.v0w, sidx, (double2 *)out_dev);
    else
        hipLaunchKernelGGL(k_vis_taps<float2>, dim3(64), dim3(256), 0, s, (const float2 *)c->taps, lay, pl.jp,
                           pl.u0w, pl.v0w, sidx, (float2 *)out_dev);
    return hipGetLastError();
}

hipError_t run_plane_taps(wsp_ctx *c, int64_t sidx, void *out_dev, hipStream_t s) {
    const Plan &pl = c->plan;
    hipLaunchKernelGGL(k_plane_vis_taps, dim3(64), dim3(256), 0, s, pl.ux, pl.vx, pl.weff, pl.jp,
                       pl.plane_off, pl.n_pairs, c->g.plane_inv_dw, (const float4 *)c->taps,
                       (float)c->g.plane_inv_dq, sidx, (float2 *)out_dev);
    return hipGetLastError();
}

}  // namespace wsp
