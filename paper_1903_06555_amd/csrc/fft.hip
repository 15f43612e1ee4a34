// F and F^dagger of the operator (Eqs. (4), (7)) as LDS-resident transforms
// fused with the image-side steps, for grids of G = 2^m cells a side
// (64 <= G <= 8192) and N <= G / 2 pixels.
//
// The 2-D DFT of the zero-padded image is computed as G-point transforms
// along V (grid rows) for every pixel column, then along U for every grid
// row.  Each transform runs in one workgroup, entirely in LDS: G/16 threads,
// 16 points per thread, Stockham autosort passes of radix 16 (and one of
// radix 2, 4 or 8 for the remaining factor), in natural order in and out.
// Because a workgroup holds a whole transform, the steps around it fuse
// into the same kernel:
//   forward: S~_k, Z and the V transform of every stack from one read of an
//            image column (k_fft_v_fwd); only the grid rows that hold work
//            items are kept (a pixel's used rows contiguous), and read
//            across pixels to be transformed along U into the grid tiles
//            that hold work items (k_fft_u_fwd);
//   inverse: the U transform of each used grid row, reading only its used
//            tiles and keeping the N columns that Z^dagger does not discard,
//            stored transposed (k_fft_u_inv); then the V transform per pixel
//            column with Z^dagger, S~_k^dagger, Re and the sum over stacks
//            (k_fft_v_inv).
// Against two library passes over the whole padded grid, with separate
// taper, transpose and crop passes, this touches only the used rows and
// tiles and never materialises the padding: where half of a transform's
// input is zero (Z's padding), its first pass reads only the other half.
#include <cmath>
#include <vector>

#include "wsp_devmath.h"
#include "wsp_image.h"

namespace wsp {

namespace {

constexpr int kPerThread = 16;  // points per thread (radix-16 passes)
constexpr int kPix = 8;         // pixels per thread along a column (N <= G / 2)
constexpr int kURows = 2;       // grid rows per block of the forward U pass (the adjoint U pass takes pairs too)
constexpr int kTT = 64;         // transpose tile

// LDS slot of point i: one pad slot after every 16 points, so that the
// strided writes of the first passes spread over the banks
__device__ __forceinline__ int lds_pos(int i) { return i + (i >> 4); }

// bit reversal of x over log2(R) bits
template <int R>
__host__ __device__ constexpr int bit_reverse(int x) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (x & 1);
        x >>= 1;
    }
    return r;
}

// cos and sin of 2 pi m / 16, m = 0 .. 7
constexpr double kCos16[8] = {1.0,
                              0.92387953251128675613,
                              0.70710678118654752440,
                              0.38268343236508977173,
                              0.0,
                              -0.38268343236508977173,
                              -0.70710678118654752440,
                              -0.92387953251128675613};
constexpr double kSin16[8] = {0.0,
                              0.38268343236508977173,
                              0.70710678118654752440,
                              0.92387953251128675613,
                              1.0,
                              0.92387953251128675613,
                              0.70710678118654752440,
                              0.38268343236508977173};

// b e^{-+2 pi i m / 16} (minus: forward, plus: inverse); m is a constant
// after unrolling, so the trivial factors cost nothing
template <bool kInv, typename C>
__device__ __forceinline__ C rot16(C b, int m) {
    using T = decltype(b.x);
    C o;
    if (m == 0) return b;
    if (m == 4) {
        if (kInv) {
            o.x = -b.y;
            o.y = b.x;
        } else {
            o.x = b.y;
            o.y = -b.x;
        }
        return o;
    }
    const T c = (T)kCos16[m], sn = kInv ? (T)kSin16[m] : (T)-kSin16[m];
    o.x = b.x * c - b.y * sn;
    o.y = b.x * sn + b.y * c;
    return o;
}

// In-register DFT of R points (R = 2, 4, 8, 16): radix-2 decimation in time
// over bit-reversed inputs, natural order out.
template <bool kInv, int R, typename C>
__device__ __forceinline__ void dft_reg(C *v) {
    C t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[bit_reverse<R>(i)] = v[i];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i0 = 0; i0 < R; i0 += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const C a = t[i0 + k];
                const C b = rot16<kInv>(t[i0 + k + len / 2], k * (16 / len));
                t[i0 + k].x = a.x + b.x;
                t[i0 + k].y = a.y + b.y;
                t[i0 + k + len / 2].x = a.x - b.x;
                t[i0 + k + len / 2].y = a.y - b.y;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// One Stockham pass of radix R over N points in LDS, after Ns points have
// been combined: butterfly j (k = j mod Ns) takes x[j + t N/R], t < R,
// twiddled by e^{-+2 pi i t k / (Ns R)}, and writes its R outputs to
// (j - k) R + k + t Ns.  Each of the N/16 threads runs 16/R butterflies; all
// reads finish before any write (in place).  The twiddles of the pass sit at
// tw[Ns - 16 + (t - 1) Ns + k] (every earlier pass has radix 16), so that
// neighbouring butterflies read neighbouring entries.
template <int R, bool kInv, int N, int Ns, typename C>
__device__ __forceinline__ void stockham_pass(C *sm, const C *__restrict__ tw, int tid) {
    constexpr int B = kPerThread / R, T = N / kPerThread, NR = N / R;
    C v[B][R];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * T;
        const int k = j & (Ns - 1);
        // when NR is a multiple of 16 the padded slots are j's plus constants
        if constexpr (NR % 16 == 0) {
            const C *src = sm + lds_pos(j);
#pragma unroll
            for (int t = 0; t < R; ++t) v[b][t] = src[t * (NR + NR / 16)];
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) v[b][t] = sm[lds_pos(j + t * NR)];
        }
        if constexpr (Ns > 1) {
            const C *twk = tw + (Ns - 16) + k;
#pragma unroll
            for (int t = 1; t < R; ++t) {
                C w = twk[(t - 1) * Ns];
                if (kInv) w.y = -w.y;
                v[b][t] = cmul(v[b][t], w);
            }
        }
        dft_reg<kInv, R>(v[b]);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = tid + b * T;
        const int k = j & (Ns - 1);
        const int base = (j - k) * R + k;
        if constexpr (Ns % 16 == 0) {
            C *dst = sm + lds_pos(base);
#pragma unroll
            for (int t = 0; t < R; ++t) dst[t * (Ns + Ns / 16)] = v[b][t];
        } else {
#pragma unroll
            for (int t = 0; t < R; ++t) sm[lds_pos(base + t * Ns)] = v[b][t];
        }
    }
    __syncthreads();
}

// The first pass (radix 16, nothing combined yet) when the inputs in
// [N/4, 3N/4) are zero and not read: butterfly j's inputs t = 4 .. 11 are
// then zero, so its 16-point DFT splits (decimation in frequency) into two
// 8-point DFTs of y_s = x_s + x_{s+8} and z_s = (x_s - x_{s+8}) e^{-+2 pi i s/16},
// of which only one term is nonzero: X_{2m} = DFT8(y)_m, X_{2m+1} = DFT8(z)_m.
template <bool kInv, int N, typename C>
__device__ __forceinline__ void first_pass_half(C *sm, int tid) {
    constexpr int NR = N / 16;
    const int j = tid;
    C y[8], z[8];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        y[s] = sm[lds_pos(j + s * NR)];
        z[s] = rot16<kInv>(y[s], s);
    }
#pragma unroll
    for (int s = 4; s < 8; ++s) {
        y[s] = sm[lds_pos(j + (s + 8) * NR)];
        z[s] = rot16<kInv>(y[s], s);
        z[s].x = -z[s].x;
        z[s].y = -z[s].y;
    }
    dft_reg<kInv, 8>(y);
    dft_reg<kInv, 8>(z);
    __syncthreads();
    C *dst = sm + lds_pos(16 * j);  // 16 j .. 16 j + 15 share one pad slot offset
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        dst[2 * m] = y[m];
        dst[2 * m + 1] = z[m];
    }
    __syncthreads();
}

template <int kLog, bool kInv, int kPass, typename C>
__device__ __forceinline__ void fft_passes(C *sm, const C *__restrict__ tw, int tid) {
    constexpr int N = 1 << kLog, Ns = 1 << (4 * kPass);
    if constexpr (Ns * 16 <= N) {
        stockham_pass<16, kInv, N, Ns>(sm, tw, tid);
        fft_passes<kLog, kInv, kPass + 1>(sm, tw, tid);
    } else if constexpr (Ns < N) {
        stockham_pass<N / Ns, kInv, N, Ns>(sm, tw, tid);
    }
}

// Unnormalised 2^kLog-point DFT (forward e^{-2 pi i ...}, inverse e^{+...})
// of the points in sm, in place, by the 2^kLog / 16 threads of the block.
// The caller synchronises between filling sm and the call.
template <int kLog, bool kInv, typename C>
__device__ __forceinline__ void lds_fft(C *sm, const C *__restrict__ tw, int tid) {
    fft_passes<kLog, kInv, 0>(sm, tw, tid);
}

// The same transform when the points in [N/4, 3N/4) are zero: they need not
// be stored (a zero-padded half, as Z leaves it), and the first pass does
// half the work.
template <int kLog, bool kInv, typename C>
__device__ __forceinline__ void lds_fft_half(C *sm, const C *__restrict__ tw, int tid) {
    first_pass_half<kInv, 1 << kLog>(sm, tid);
    fft_passes<kLog, kInv, 1>(sm, tw, tid);
}

// x, hidden from the optimiser: inside the per-stack loops, the transform's
// addresses are recomputed from it on every stack instead of being hoisted
// out of the loop and held in registers across it
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Grid tiles that hold work items, one bit per 64 x 64 tile: row ty of
// stack k is kTileWords words at (k G/64 + ty) kTileWords.  F fills only
// these tiles (the sparse steps read nothing else) and F^dagger reads only
// these (every other cell is zero).
template <int G>
constexpr int kTileWords = (G / kTile + 63) / 64;

// A grid row's tile bits, read once (G <= 8192: at most two words).
template <int G>
struct TileRow {
    uint64_t w[kTileWords<G>];
    __device__ __forceinline__ explicit TileRow(const uint64_t *__restrict__ trow) {
#pragma unroll
        for (int i = 0; i < kTileWords<G>; ++i) w[i] = trow[i];
    }
    // whether grid column U lies in a used tile (uniform over each 64
    // consecutive U, so over a wavefront)
    __device__ __forceinline__ bool used(int U) const {
        const int tx = U / kTile;
        return (w[tx >> 6] >> (tx & 63)) & 1ull;
    }
    // The same with the word picked by selects.  In the adjoint U pass, which
    // loads two rows, the indexed form above is compiled to an array in
    // scratch memory; in the forward U pass's stores it is the faster form
    // (2.85 against 3.09 ms measured with selects).
    __device__ __forceinline__ bool used_sel(int U) const {
        const int tx = U / kTile;
        uint64_t word = w[0];
#pragma unroll
        for (int i = 1; i < kTileWords<G>; ++i) word = (tx >> 6) == i ? w[i] : word;
        return (word >> (tx & 63)) & 1ull;
    }
};

// grid row of used-row slot rr: rows [0, rows_lo), then [G - rows_hi, G)
__device__ __forceinline__ int used_row(int rr, const Geom &g) {
    return rr < g.rows_lo ? rr : g.G - g.rows_hi + (rr - g.rows_lo);
}

// Work index of block b when the blocks of neighbouring indices should run
// on one XCD (blocks are dealt to the 8 XCDs in turn): XCD b mod 8 takes the
// (b mod 8)-th contiguous eighth of [0, n), in order.  A kernel whose blocks
// each store a column of a matrix (8- or 16-byte elements a row apart) then
// fills the cache lines of its neighbours in the same L2, which writes them
// back whole.  The grid has 8 ceil(n / 8) blocks; -1 past n.
__device__ __forceinline__ int xcd_index(int b, int n) {
    const int per = (n + 7) / 8;
    const int idx = (b % 8) * per + b / 8;
    return idx < n ? idx : -1;
}

// Forward, first half.  Block: pixel column i.  For every stack k of [k0, k1),
// sm[V] = S~_k Z x along column i (zero where Z pads), transformed along V;
// the used rows go to hp[k][i][rr] (rows ld apart).  Pixel j of the column
// is thread j mod T's (q = j / T < 8, as N <= G / 2).
template <bool kFP64, int kLog>
__global__ __launch_bounds__(1 << (kLog - 4), kFP64 ? 2 : 4) void k_fft_v_fwd(
    const typename Types<kFP64>::R *__restrict__ imageT, typename Types<kFP64>::C *__restrict__ hp,
    const typename Types<kFP64>::C *__restrict__ tw, const double *__restrict__ centres, Geom g, int n_used, int ld,
    int k0, int k1) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int G = 1 << kLog, T = G / kPerThread;
    __shared__ C sm[G + G / 16];
    const int i = blockIdx.x, tid = threadIdx.x;
    const int n = g.n, h = n / 2;
    R av[kPix];
    double nm[kPix];
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int j = tid + q * T;
        av[q] = 0;
        nm[q] = 0.0;
        if (j < n) {
            double amp, nm1;
            pixel_factors(j, i, g, &amp, &nm1);
            av[q] = (R)((double)imageT[(int64_t)i * n + j] * amp);
            nm[q] = nm1;
        }
    }
    C zero;
    zero.x = 0;
    zero.y = 0;
    for (int k = k0; k < k1; ++k) {
        const double ck = centres[k];
#pragma unroll
        for (int q = 0; q < kPix; ++q) {
            const int j = tid + q * T;
            if (j < n) {
                R sn, cs;
                rev_sincos<kFP64>(reduce_rev(-ck * nm[q]), &sn, &cs);
                C z;
                z.x = av[q] * cs;
                z.y = av[q] * sn;
                sm[lds_pos(padded_of(j, g))] = z;
            }
        }
        // zeros where Z pads, except [G/4, 3G/4), which the first pass skips
        for (int V = h + tid; V < G / 4; V += T) sm[lds_pos(V)] = zero;
        for (int V = 3 * (G / 4) + tid; V < G - h; V += T) sm[lds_pos(V)] = zero;
        __syncthreads();
        lds_fft_half<kLog, false>(sm, tw, opaque(tid));
        C *dst = hp + ((int64_t)k * n + i) * ld;
        for (int rr = tid; rr < n_used; rr += T) dst[rr] = sm[lds_pos(used_row(rr, g))];
        __syncthreads();
    }
}

// The kPix pixel values of one row of n that thread tid holds (i = tid + q T).
template <int T, typename C>
__device__ __forceinline__ void fetch_pixels(C (&pre)[kPix], const C *__restrict__ src, int n, int tid) {
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int i = tid + q * T;
        pre[q].x = 0;
        pre[q].y = 0;
        if (i < n) pre[q] = src[i];
    }
}

// The kPerThread cells U = tid + q T of grid row V of stack k: its used
// tiles' values, zero elsewhere.
template <int G, typename C>
__device__ __forceinline__ void fetch_row(C (&pre)[kPerThread], const C *__restrict__ grids,
                                          const uint64_t *__restrict__ tiles, int k, int V, int tid) {
    constexpr int T = G / kPerThread;
    const C *src = grids + ((int64_t)k * G + V) * G;
    const TileRow<G> trow(tiles + ((int64_t)k * (G / kTile) + V / kTile) * kTileWords<G>);
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int U = tid + q * T;
        pre[q].x = 0;
        pre[q].y = 0;
        if (trow.used_sel(U)) pre[q] = src[U];
    }
}

// The kURows consecutive used rows rr0 .. of the kPix pixels i = tid + q T
// that thread tid holds (contiguous in hp; ld and rr0 are multiples of
// kURows, so for FP32 they are one aligned 16-byte load).
template <int T>
__device__ __forceinline__ void fetch_rows(float2 (&pre)[kPix][kURows], const float2 *__restrict__ src, int ld,
                                           int n, int tid) {
    static_assert(kURows == 2, "one 16-byte load per pixel");
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int i = tid + q * T;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < n) a = *(const float4 *)(src + (int64_t)i * ld);
        pre[q][0] = make_float2(a.x, a.y);
        pre[q][1] = make_float2(a.z, a.w);
    }
}
template <int T>
__device__ __forceinline__ void fetch_rows(double2 (&pre)[kPix][kURows], const double2 *__restrict__ src, int ld,
                                           int n, int tid) {
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int i = tid + q * T;
#pragma unroll
        for (int r = 0; r < kURows; ++r) {
            pre[q][r] = make_double2(0.0, 0.0);
            if (i < n) pre[q][r] = src[(int64_t)i * ld + r];
        }
    }
}

// pre[r] with r uniform but not a constant (selects, not a dynamically
// indexed register array)
template <typename C>
__device__ __forceinline__ C pick_row(const C (&pre)[kURows], int r) {
    C v = pre[0];
#pragma unroll
    for (int s = 1; s < kURows; ++s) {
        v.x = r == s ? pre[s].x : v.x;
        v.y = r == s ? pre[s].y : v.y;
    }
    return v;
}

// Forward, second half.  Block: kURows consecutive used-row slots rr of
// stack k (blocks in xcd_index order over the row groups of stacks
// [k0, k0 + nk)).  Row V(rr) of the padded transform, from hp[k][i][rr] at
// the pixel columns (zero where Z pads), transformed along U into the used
// tiles of the grid.  A pixel's kURows rows are contiguous in hp, so each
// thread loads the group's rows of its pixels at once; the groups that
// share cache lines run on one XCD at about the same time and find them in
// its L2.
template <bool kFP64, int kLog>
__global__ __launch_bounds__(1 << (kLog - 4), kFP64 ? 2 : 4) void k_fft_u_fwd(
    const typename Types<kFP64>::C *__restrict__ hp, typename Types<kFP64>::C *__restrict__ grids,
    const typename Types<kFP64>::C *__restrict__ tw, const uint64_t *__restrict__ tiles, Geom g, int n_used,
    int ld, int k0, int nk) {
    using C = typename Types<kFP64>::C;
    constexpr int G = 1 << kLog, T = G / kPerThread;
    __shared__ C sm[G + G / 16];
    const int groups = (n_used + kURows - 1) / kURows;
    const int grp = xcd_index(blockIdx.x, nk * groups);
    if (grp < 0) return;  // uniform over the block
    const int k = k0 + grp / groups, rr0 = (grp % groups) * kURows, tid = threadIdx.x;
    const int n = g.n, h = n / 2;
    const int rr_end = rr0 + kURows < n_used ? rr0 + kURows : n_used;
    C zero;
    zero.x = 0;
    zero.y = 0;
    C pre[kPix][kURows];
    fetch_rows<T>(pre, hp + (int64_t)k * n * ld + rr0, ld, n, tid);
    for (int rr = rr0; rr < rr_end; ++rr) {
        const int t = opaque(tid);
#pragma unroll
        for (int q = 0; q < kPix; ++q) {
            const int i = t + q * T;
            if (i < n) sm[lds_pos(padded_of(i, g))] = pick_row(pre[q], rr - rr0);
        }
        for (int U = h + t; U < G / 4; U += T) sm[lds_pos(U)] = zero;
        for (int U = 3 * (G / 4) + t; U < G - h; U += T) sm[lds_pos(U)] = zero;
        __syncthreads();
        lds_fft_half<kLog, false>(sm, tw, t);
        const int V = used_row(rr, g);
        C *dst = grids + ((int64_t)k * G + V) * G;
        const TileRow<G> trow(tiles + ((int64_t)k * (G / kTile) + V / kTile) * kTileWords<G>);
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int U = t + q * T;
            if (trow.used(U)) dst[U] = sm[lds_pos(U)];
        }
        __syncthreads();  // sm is refilled for the next row
    }
}

// A pixel's values of two neighbouring used rows, stored together (16 bytes
// for FP32: ld and rr0 are even)
__device__ __forceinline__ void store_pair(float2 *dst, float2 a, float2 b) {
    *(float4 *)dst = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(double2 *dst, double2 a, double2 b) {
    dst[0] = a;
    dst[1] = b;
}

// Inverse, first half.  Block: used-row slots rr0, rr0 + 1 of stack k
// (blocks in xcd_index order over the row pairs of stacks [k0, k0 + nk)).
// Grid rows V(rr) (their used tiles; zero elsewhere) transformed back along
// U, the second row's loads in flight during the first transform; the N
// pixel columns go to rows rr0, rr0 + 1 of hp[k][i][rr] (the layout the V
// pass reads), a pixel's two values in one store.
template <bool kFP64, int kLog>
__global__ __launch_bounds__(1 << (kLog - 4), kFP64 ? 2 : 4) void k_fft_u_inv(
    const typename Types<kFP64>::C *__restrict__ grids, typename Types<kFP64>::C *__restrict__ hp,
    const typename Types<kFP64>::C *__restrict__ tw, const uint64_t *__restrict__ tiles, Geom g, int n_used,
    int ld, int k0, int nk) {
    using C = typename Types<kFP64>::C;
    constexpr int G = 1 << kLog, T = G / kPerThread;
    __shared__ C sm[G + G / 16];
    const int pairs = (n_used + 1) / 2;
    const int grp = xcd_index(blockIdx.x, nk * pairs);
    if (grp < 0) return;  // uniform over the block
    const int k = k0 + grp / pairs, rr0 = (grp % pairs) * 2, tid = threadIdx.x;
    const bool two = rr0 + 1 < n_used;  // uniform
    const int n = g.n;
    C v[kPerThread];  // all loads in flight before the LDS stores
    fetch_row<G>(v, grids, tiles, k, used_row(rr0, g), tid);
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) sm[lds_pos(tid + q * T)] = v[q];
    if (two) fetch_row<G>(v, grids, tiles, k, used_row(rr0 + 1, g), tid);
    __syncthreads();
    lds_fft<kLog, true>(sm, tw, tid);
    C first[kPix];
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int i = tid + q * T;
        first[q] = v[0];  // defined for every q (unused past n)
        if (i < n) first[q] = sm[lds_pos(padded_of(i, g))];
    }
    C *dst = hp + (int64_t)k * n * ld + rr0;
    if (!two) {
#pragma unroll
        for (int q = 0; q < kPix; ++q) {
            const int i = tid + q * T;
            if (i < n) dst[(int64_t)i * ld] = first[q];
        }
        return;  // uniform over the block
    }
    __syncthreads();  // sm is refilled for the second row
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) sm[lds_pos(tid + q * T)] = v[q];
    __syncthreads();
    lds_fft<kLog, true>(sm, tw, tid);
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int i = tid + q * T;
        if (i < n) store_pair(dst + (int64_t)i * ld, first[q], sm[lds_pos(padded_of(i, g))]);
    }
}

// Inverse, second half.  Block: pixel column i.  For every stack k, the
// column hp[k][i][rr] placed at its used rows (zero elsewhere: rows without
// work items hold no data) and transformed back along V; Z^dagger keeps the
// pixel rows, S~_k^dagger and Re weight them, and the stacks are summed
// (FP64 sum).  Output transposed: imageT[i][j].  kHalf: the used rows all
// lie outside [G/4, 3G/4), whose points the first pass then skips.
template <bool kFP64, int kLog, bool kHalf>
__global__ __launch_bounds__(1 << (kLog - 4), kFP64 ? 2 : 4) void k_fft_v_inv(
    const typename Types<kFP64>::C *__restrict__ hp, typename Types<kFP64>::R *__restrict__ imageT,
    const typename Types<kFP64>::C *__restrict__ tw, const double *__restrict__ centres, Geom g, int n_used,
    int ld) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    constexpr int G = 1 << kLog, T = G / kPerThread;
    __shared__ C sm[G + G / 16];
    const int i = blockIdx.x, tid = threadIdx.x;
    const int n = g.n;
    double nm[kPix], acc[kPix];
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int j = tid + q * T;
        nm[q] = 0.0;
        acc[q] = 0.0;
        if (j < n) {
            double amp;
            pixel_factors(j, i, g, &amp, &nm[q]);
        }
    }
    C zero;
    zero.x = 0;
    zero.y = 0;
    // the first kPix T used rows of the next stack's column are loaded while
    // the current stack is transformed
    C pre[kPix];
    fetch_pixels<T>(pre, hp + (int64_t)i * ld, n_used, tid);
    for (int k = 0; k < g.n_stacks; ++k) {
        const int t = opaque(tid);
        const C *src = hp + ((int64_t)k * n + i) * ld;
#pragma unroll
        for (int q = 0; q < kPix; ++q) {
            const int rr = t + q * T;
            if (rr < n_used) sm[lds_pos(used_row(rr, g))] = pre[q];
        }
        for (int rr = t + kPix * T; rr < n_used; rr += T) sm[lds_pos(used_row(rr, g))] = src[rr];
        if constexpr (kHalf) {
            for (int V = g.rows_lo + t; V < G / 4; V += T) sm[lds_pos(V)] = zero;
            for (int V = 3 * (G / 4) + t; V < G - g.rows_hi; V += T) sm[lds_pos(V)] = zero;
        } else {
            for (int V = g.rows_lo + t; V < G - g.rows_hi; V += T) sm[lds_pos(V)] = zero;
        }
        if (k + 1 < g.n_stacks) fetch_pixels<T>(pre, hp + ((int64_t)(k + 1) * n + i) * ld, n_used, tid);
        __syncthreads();
        if constexpr (kHalf) lds_fft_half<kLog, true>(sm, tw, t);
        else lds_fft<kLog, true>(sm, tw, t);
        const double ck = centres[k];
#pragma unroll
        for (int q = 0; q < kPix; ++q) {
            const int j = tid + q * T;
            if (j < n) {
                R sn, cs;
                rev_sincos<kFP64>(reduce_rev(-ck * nm[q]), &sn, &cs);
                const C z = sm[lds_pos(padded_of(j, g))];
                // Re(z conj(s_k)) with s_k = amp e^{2 pi i rev}; amp after the sum
                acc[q] += (double)(z.x * cs + z.y * sn);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int j = tid + q * T;
        if (j < n) {
            double amp, nm1;
            pixel_factors(j, i, g, &amp, &nm1);
            imageT[(int64_t)i * n + j] = (R)(amp * acc[q]);
        }
    }
}

// Clear the used tiles of the grids before the adjoint's sparse step (which
// adds into them).  Block: one tile of the list (keys stack | ty | tx).
template <typename C>
__global__ __launch_bounds__(256) void k_zero_tiles(C *grids, const uint32_t *__restrict__ list, int tile_bits,
                                                    int G) {
    const uint32_t key = list[blockIdx.x];
    const uint32_t tmask = (1u << tile_bits) - 1;
    const int tx = (int)(key & tmask), ty = (int)((key >> tile_bits) & tmask), k = (int)(key >> (2 * tile_bits));
    C *dst = grids + ((int64_t)k * G + (int64_t)ty * kTile) * G + (int64_t)tx * kTile;
    C zero;
    zero.x = 0;
    zero.y = 0;
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) dst[(int64_t)(e / kTile) * G + (e % kTile)] = zero;
}

// dst[b][c][r] = src[b][r][c] for a batch of rows x cols matrices (64 x 64
// tiles through LDS: coalesced reads and writes; each thread's 16 loads are
// all issued before the LDS stores).  Block: (column tile, row tile, batch).
template <typename E>
__global__ __launch_bounds__(256) void k_transpose_batch(const E *__restrict__ src, E *__restrict__ dst,
                                                         int rows, int cols) {
    constexpr int kPer = kTT * kTT / 256;
    __shared__ E s_t[kTT][kTT + 1];
    const int c0 = blockIdx.x * kTT, r0 = blockIdx.y * kTT;
    const int64_t off = (int64_t)blockIdx.z * rows * cols;
    const int c = threadIdx.x % kTT, rq = threadIdx.x / kTT;  // rows rq, rq + 4, ...
    E v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int r = rq + 4 * q;
        v[q] = E{};
        if (r0 + r < rows && c0 + c < cols) v[q] = src[off + (int64_t)(r0 + r) * cols + c0 + c];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) s_t[rq + 4 * q][c] = v[q];
    __syncthreads();
    // now c indexes rows of the source (contiguous in dst), rq + 4 q its columns
#pragma unroll
    for (int q = 0; q < kPer; ++q) v[q] = s_t[c][rq + 4 * q];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int cc = rq + 4 * q;
        if (r0 + c < rows && c0 + cc < cols) dst[off + (int64_t)(c0 + cc) * rows + r0 + c] = v[q];
    }
}

template <typename E>
void transpose_batch(const E *src, E *dst, int rows, int cols, int batch, hipStream_t s) {
    const dim3 gd((unsigned)((cols + kTT - 1) / kTT), (unsigned)((rows + kTT - 1) / kTT), (unsigned)batch);
    hipLaunchKernelGGL(k_transpose_batch<E>, gd, dim3(256), 0, s, src, dst, rows, cols);
}

template <bool kFP64>
constexpr size_t lds_bytes(int G) {
    return sizeof(typename Types<kFP64>::C) * (size_t)(G + G / 16);
}

}  // namespace

bool fft_lds_fits(int G, int n, bool fp64, int device) {
    if (G < 64 || G > 8192 || (G & (G - 1)) != 0) return false;
    if (2 * n > G) return false;  // at most kPix pixels per thread
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return false;
    const size_t need = fp64 ? lds_bytes<true>(G) : lds_bytes<false>(G);
    return need <= (size_t)lds;
}

// Twiddles of the Stockham passes after the first (fewer than G entries):
// pass (radix R, Ns points combined before it) holds e^{-2 pi i t k / (Ns R)}
// for t in [1, R), k in [0, Ns) at Ns - 16 + (t - 1) Ns + k, computed in
// FP64 and rounded to the operator's complex type.
hipError_t fft_lds_twiddles(int G, bool fp64, void *dev) {
    std::vector<double> w(2 * (size_t)G, 0.0);
    for (int Ns = 16; Ns < G;) {
        const int R = Ns * 16 <= G ? 16 : G / Ns;
        for (int t = 1; t < R; ++t) {
            for (int k = 0; k < Ns; ++k) {
                const size_t e = (size_t)(Ns - 16) + (size_t)(t - 1) * Ns + k;
                // t k / (Ns R) revolutions, reduced to [0, 1) exactly (powers of two)
                const double rev = (double)((int64_t)t * k % ((int64_t)Ns * R)) / ((double)Ns * R);
                w[2 * e] = std::cos(2.0 * M_PI * rev);
                w[2 * e + 1] = -std::sin(2.0 * M_PI * rev);
            }
        }
        Ns *= R;
    }
    if (fp64) return hipMemcpy(dev, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice);
    std::vector<float> f(w.size());
    for (size_t k = 0; k < w.size(); ++k) f[k] = (float)w[k];
    return hipMemcpy(dev, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice);
}

// Row stride of hp: the used rows, rounded up to whole row groups of the
// forward U pass.
static int hp_ld(const Geom &g) { return (g.rows_lo + g.rows_hi + kURows - 1) / kURows * kURows; }

static size_t hp_bytes(const Geom &g, bool fp64) {
    return ((size_t)g.n_stacks * g.n * hp_ld(g) * (fp64 ? 16 : 8) + 255) & ~(size_t)255;
}

// Scratch of the LDS transforms: hp [K][N][ld] (a pixel column's used rows,
// between the two passes of either direction), then the transposed image
// imageT [N][N] (the forward's input, the adjoint's output).
size_t fft_lds_scratch_bytes(const Geom &g, bool fp64) {
    return hp_bytes(g, fp64) + (size_t)g.n * g.n * (fp64 ? 8 : 4);
}

namespace {

template <bool kFP64>
struct LdsBuffers {
    typename Types<kFP64>::C *hp;
    typename Types<kFP64>::R *imageT;
};

template <bool kFP64>
LdsBuffers<kFP64> lds_buffers(const Geom &g, void *scratch) {
    using C = typename Types<kFP64>::C;
    const size_t half = hp_bytes(g, kFP64);
    LdsBuffers<kFP64> b;
    b.hp = (C *)scratch;
    b.imageT = (typename Types<kFP64>::R *)((char *)scratch + half);
    return b;
}

// Launch F<kLog>::run with the grid size as a template constant.
template <template <int> class F, typename... A>
void by_size(int G, A... args) {
    switch (G) {
        case 64: F<6>::run(args...); break;
        case 128: F<7>::run(args...); break;
        case 256: F<8>::run(args...); break;
        case 512: F<9>::run(args...); break;
        case 1024: F<10>::run(args...); break;
        case 2048: F<11>::run(args...); break;
        case 4096: F<12>::run(args...); break;
        case 8192: F<13>::run(args...); break;
        default: break;  // not reached: fft_lds_fits admits only these sizes
    }
}

template <bool kFP64>
struct Launch {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    template <int kLog>
    struct Forward {
        static void run(const Geom &g, C *grids, LdsBuffers<kFP64> b, const C *tw, const uint64_t *tiles,
                        const double *centres, int k0, int k1, hipStream_t s) {
            const int used = g.rows_lo + g.rows_hi, nk = k1 - k0, ld = hp_ld(g);
            const dim3 bd(1u << (kLog - 4));
            hipLaunchKernelGGL((k_fft_v_fwd<kFP64, kLog>), dim3((unsigned)g.n), bd, 0, s, (const R *)b.imageT,
                               b.hp, tw, centres, g, used, ld, k0, k1);
            const int64_t groups = (int64_t)nk * ((used + kURows - 1) / kURows);
            hipLaunchKernelGGL((k_fft_u_fwd<kFP64, kLog>), dim3(8u * (unsigned)((groups + 7) / 8)), bd, 0, s,
                               (const C *)b.hp, grids, tw, tiles, g, used, ld, k0, nk);
        }
    };
    template <int kLog>
    struct Inverse {
        static void run(const Geom &g, const C *grids, LdsBuffers<kFP64> b, const C *tw, const uint64_t *tiles,
                        int k0, int k1, hipStream_t s) {
            const int used = g.rows_lo + g.rows_hi, nk = k1 - k0;
            const int64_t pairs = (int64_t)nk * ((used + 1) / 2);
            hipLaunchKernelGGL((k_fft_u_inv<kFP64, kLog>), dim3(8u * (unsigned)((pairs + 7) / 8)),
                               dim3(1u << (kLog - 4)), 0, s, grids, b.hp, tw, tiles, g, used, hp_ld(g), k0,
                               nk);
        }
    };
    template <int kLog>
    struct ImageOut {
        static void run(const Geom &g, R *image, LdsBuffers<kFP64> b, const C *tw, const double *centres,
                        hipStream_t s) {
            const int used = g.rows_lo + g.rows_hi;
            // kHalf: used rows all outside [G/4, 3G/4), so the first pass skips that half
            const bool half = g.rows_lo <= (1 << kLog) / 4 && g.rows_hi <= (1 << kLog) / 4;
            if (half)
                hipLaunchKernelGGL((k_fft_v_inv<kFP64, kLog, true>), dim3((unsigned)g.n), dim3(1u << (kLog - 4)),
                                   0, s, (const C *)b.hp, b.imageT, tw, centres, g, used,
                                   hp_ld(g));
            else
                hipLaunchKernelGGL((k_fft_v_inv<kFP64, kLog, false>), dim3((unsigned)g.n), dim3(1u << (kLog - 4)),
                                   0, s, (const C *)b.hp, b.imageT, tw, centres, g, used,
                                   hp_ld(g));
            transpose_batch<R>(b.imageT, image, g.n, g.n, 1, s);
        }
    };
};

}  // namespace

// Forward, image side: the image transposed (pixel columns contiguous).
template <bool kFP64>
hipError_t fft_lds_image_in(const Geom &g, const void *image, void *scratch, hipStream_t s) {
    using R = typename Types<kFP64>::R;
    const LdsBuffers<kFP64> b = lds_buffers<kFP64>(g, scratch);
    transpose_batch<R>((const R *)image, b.imageT, g.n, g.n, 1, s);
    return hipGetLastError();
}

// Forward: S~_k, Z and F of stacks [k0, k1) into the used tiles of the grids.
template <bool kFP64>
hipError_t fft_lds_forward(const Geom &g, void *grids, void *scratch, const void *tw, const uint64_t *tiles,
                           const double *centres, int k0, int k1, hipStream_t s) {
    using C = typename Types<kFP64>::C;
    by_size<Launch<kFP64>::template Forward>(g.G, g, (C *)grids, lds_buffers<kFP64>(g, scratch), (const C *)tw,
                                             tiles, centres, k0, k1, s);
    return hipGetLastError();
}

// Inverse, grid side: F^dagger along U of the used rows of stacks [k0, k1),
// transposed.
template <bool kFP64>
hipError_t fft_lds_inverse(const Geom &g, const void *grids, void *scratch, const void *tw, const uint64_t *tiles,
                           int k0, int k1, hipStream_t s) {
    using C = typename Types<kFP64>::C;
    by_size<Launch<kFP64>::template Inverse>(g.G, g, (const C *)grids, lds_buffers<kFP64>(g, scratch),
                                             (const C *)tw, tiles, k0, k1, s);
    return hipGetLastError();
}

// Inverse, image side: F^dagger along V, Z^dagger, S~_k^dagger, Re and the
// sum over stacks, into the image.
template <bool kFP64>
hipError_t fft_lds_image_out(const Geom &g, void *image, void *scratch, const void *tw, const double *centres,
                             hipStream_t s) {
    using R = typename Types<kFP64>::R;
    using C = typename Types<kFP64>::C;
    by_size<Launch<kFP64>::template ImageOut>(g.G, g, (R *)image, lds_buffers<kFP64>(g, scratch), (const C *)tw,
                                              centres, s);
    return hipGetLastError();
}

template <bool kFP64>
hipError_t fft_lds_zero_tiles(const Geom &g, void *grids, const uint32_t *list, int n_tiles, int tile_bits,
                              hipStream_t s) {
    using C = typename Types<kFP64>::C;
    if (n_tiles > 0)
        hipLaunchKernelGGL(k_zero_tiles<C>, dim3((unsigned)n_tiles), dim3(256), 0, s, (C *)grids, list, tile_bits,
                           g.G);
    return hipGetLastError();
}

// One bit per used tile (see kTileWords) and the list of used tile keys,
// from the work items' tile keys (host side, at planning).
void fft_lds_tile_sets(const Geom &g, const std::vector<uint32_t> &keys, int tile_bits, std::vector<uint64_t> *bits,
                       std::vector<uint32_t> *list) {
    const int TT = g.G / kTile, W = (TT + 63) / 64;
    bits->assign((size_t)g.n_stacks * TT * W, 0ull);
    list->clear();
    const uint32_t tmask = (1u << tile_bits) - 1;
    for (uint32_t key : keys) {
        const int tx = (int)(key & tmask), ty = (int)((key >> tile_bits) & tmask), k = (int)(key >> (2 * tile_bits));
        uint64_t &w = (*bits)[((size_t)k * TT + ty) * W + (tx >> 6)];
        const uint64_t bit = 1ull << (tx & 63);
        if (!(w & bit)) list->push_back(key);
        w |= bit;
    }
}

#define WSP_FFT_LDS_INST(F64)                                                                                      \
    template hipError_t fft_lds_image_in<F64>(const Geom &, const void *, void *, hipStream_t);                   \
    template hipError_t fft_lds_forward<F64>(const Geom &, void *, void *, const void *, const uint64_t *,         \
                                             const double *, int, int, hipStream_t);                              \
    template hipError_t fft_lds_inverse<F64>(const Geom &, const void *, void *, const void *, const uint64_t *,   \
                                             int, int, hipStream_t);                                              \
    template hipError_t fft_lds_image_out<F64>(const Geom &, void *, void *, const void *, const double *,        \
                                               hipStream_t);                                                      \
    template hipError_t fft_lds_zero_tiles<F64>(const Geom &, void *, const uint32_t *, int, int, hipStream_t);
WSP_FFT_LDS_INST(false)
WSP_FFT_LDS_INST(true)
#undef WSP_FFT_LDS_INST

}  // namespace wsp
