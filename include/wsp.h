/*
 * wsp.h -- C ABI of the MI355X (gfx950) w-stacking w-projection library.
 *
 * The library applies the measurement operator of Pratley, Johnston-Hollitt &
 * McEwen (2019), "w-stacking w-projection hybrid algorithm for wide-field
 * interferometric imaging", Sec. 3.1, Eqs. (2)-(7):
 *
 *     Phi_k = W_k GC_k F Z S~_k,        Phi^dagger y = sum_k Phi_k^dagger y_k,
 *
 * with one exact w-projection kernel per visibility (the radial integral of
 * Eq. (6), evaluated by adaptive Gauss-Kronrod quadrature), w-stacks chosen by
 * the k-means iteration of Algorithm 1 (Sec. 3.2) after conjugate-symmetry
 * folding of w < 0 visibilities (Eq. (8), Sec. 3.3).
 *
 * Conventions shared by every entry point:
 *  - image: real N x N, row-major, row j <-> m_j = (j - N/2) dl, column i <->
 *    l_i = (i - N/2) dl, dl = fov / N; float32 (WSP_FP32_FP64PHASE) or
 *    float64 (WSP_FP64);
 *  - visibilities: complex, interleaved (re, im), in the caller's order;
 *    complex64 or complex128 by precision;
 *  - uvw: float64 [M][3] in wavelengths, device memory;
 *  - y = Phi x is the unnormalised operator: pixel values are Jy/pixel and no
 *    dl dm factor is applied (the paper rescales Phi by the power method);
 *  - the adjoint returns Re Phi^dagger y (the image is real, Eq. (2)).
 *  - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Every call returns a wsp_status: 0 = OK, > 0 = warning, < 0 = error.  No
 * call throws or aborts.  wsp_last_error() returns a thread-local message for
 * the last non-zero status.  A context is not thread-safe; separate contexts
 * may be used concurrently on separate streams.
 *
 * Memory ownership: wsp_set_uvw allocates the per-visibility plan (sorted
 * indices, supports, tap offsets, tile work lists; O(M) bytes) inside the
 * library and frees it in wsp_destroy.  The three large buffers -- kernel
 * taps, per-stack Fourier grids and scratch -- are owned by the caller, sized
 * by wsp_footprint and attached with wsp_bind_memory; they must stay alive
 * until wsp_destroy or the next bind.
 */
#ifndef WSP_H
#define WSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wsp_status;

#define WSP_OK 0
#define WSP_WARN_QUAD_MAXEVAL 1   /* some quadrature hit its panel cap       */
#define WSP_EINVAL -1             /* bad argument or parameter               */
#define WSP_ENOMEM_BINDING -2     /* memory not bound, or a buffer too small */
#define WSP_ESUPPORT -3           /* a kernel support exceeds max_support    */
#define WSP_EHIP -4               /* HIP or hipFFT failure                   */
#define WSP_ESTATE -5             /* called out of order                     */

#define WSP_FP32_FP64PHASE 0      /* FP32 data and taps, FP64 phase arguments */
#define WSP_FP64 1                /* FP64 everywhere                          */

#define WSP_KERNELS_EXACT 0       /* one set of J_p x J_p taps per visibility (Eq. (6))   */
#define WSP_KERNELS_PLANES 1      /* taps interpolated on the fly from 1-D w-planes     */

#define WSP_LAYOUT_AUTO 0         /* exact mode: the library's choice (contiguous runs)  */
#define WSP_LAYOUT_RUNS 1         /* each run's taps contiguous, row-major               */
#define WSP_LAYOUT_INTERLEAVED 2  /* runs of a band in groups of 64, tap k of every run
                                     of a group stored together                          */

typedef struct wsp_params {
    int32_t n;              /* image side N, even, multiple of 32                       */
    double oversample;      /* alpha; alpha*N must be an integer multiple of 64         */
    double fov_rad;         /* full field of view (direction cosine), alpha^2 fov/2 < 1 */
    int32_t kb_support;     /* J: Kaiser-Bessel support in cells, even, >= 2            */
    double kb_beta;         /* KB shape; 0 selects 2.34 J                               */
    double support_scale;   /* f >= 1: J_p = J + 2 ceil(|w - wbar| s f) (see below)     */
    int32_t n_stacks;       /* K >= 1 w-stacks                                          */
    int32_t fold_conjugate; /* 1: fold w < 0 onto w > 0 by Eq. (8)                      */
    double quad_rel_tol;    /* quadrature tolerances (the paper's value is 1e-6, Sec. 4)*/
    double quad_abs_tol;    /*   both relative to the visibility's kernel peak; the
                               smaller positive one bounds each tap's error estimate    */
    int32_t quad_max_panels;/* cap on quadrature panels per visibility (8..1024)       */
    int32_t max_support;    /* cap on J_p; larger supports give WSP_ESUPPORT            */
    int32_t precision;      /* WSP_FP32_FP64PHASE or WSP_FP64                           */
    double kmeans_tol;      /* Algorithm 1 convergence (the paper uses 1e-3, Sec. 4)    */
    int32_t kmeans_max_iter;/* iteration cap of Algorithm 1                             */
    int32_t device;         /* HIP device ordinal                                       */
    int32_t kernel_mode;    /* WSP_KERNELS_EXACT or WSP_KERNELS_PLANES (see below)      */
    double plane_dq;        /* w-plane mode: sample step in q (cells); 0 selects 1/64   */
    double plane_dw;        /* w-plane mode: plane step in |w| (wavelengths); 0: 1/16   */
    int32_t dde_support;    /* J_D: odd width of a per-visibility DDE kernel, 0 or 1 = none */
    int32_t item_taps;      /* taps per tile work item before its last entry; 0: 2^19 (a
                               tuning and test knob: small values split tiles over items) */
    int32_t band_rows;      /* exact mode: tile rows per band of the tap layout, 8 or 16;
                               0 selects 8. Results do not depend on it beyond
                               rounding order (a tuning and test knob)              */
    int32_t tap_layout;     /* exact mode: WSP_LAYOUT_* (see "Tap layouts" below)        */
} wsp_params;

/* Direction-dependent effects (Sec. 5.2, Eq. (11)).  With dde_support = J_D
 * >= 3 (odd, <= 15) every visibility's kernel becomes D_p * K_p, the discrete
 * convolution of its w-projection kernel with a separable J_D x J_D kernel
 * D_p[b, a] = d_v[p][b] d_u[p][a] given on the uv grid (a along u, b along v,
 * offsets -h .. h, h = (J_D - 1) / 2):
 *     K'_p[r, c] = sum_{a, b} d_v[p][b] d_u[p][a] K_p[r - b, c - a].
 * Supports grow to J_p' = J + 2 ceil(|w - wbar| s f) + J_D - 1 (the base rule
 * U0 = floor(u/du) - J_p'/2 + 1 is unchanged, so D is centred), and the taps
 * hold K'.  The d arrays are set with wsp_set_dde before wsp_build_kernels;
 * the convolution is applied in two 1-D passes (O(J_p'^2 J_D) per
 * visibility).  Exact kernel mode only; J_D * max J_p' complex values must
 * fit 64 KiB (WSP_ESUPPORT otherwise). */

/* Kernel modes.
 *
 * WSP_KERNELS_EXACT: wsp_build_kernels integrates Eq. (6) for every tap of
 * every visibility and stores the taps (sum_p J_p^2 complex values).
 *
 * WSP_KERNELS_PLANES (Sec. 5.1.1, bilinear interpolation between w-planes):
 * radial symmetry makes the kernel a function of the tap distance q and w
 * only, so wsp_build_kernels integrates Eq. (6) on the lattice
 * T[j, i] = K(i dq, j dw), q, w >= 0 (the pre-sampled 1-D w-planes), and
 * degrid and grid evaluate every tap on the fly by bilinear interpolation:
 * with a = |w_eff| / dw, j = floor(a), s = a - j, x = q / dq, i = floor(x),
 * t = x - i,
 *     K~ = (1 - s)[(1 - t) T[j, i] + t T[j, i+1]] + s[(1 - t) T[j+1, i] + t T[j+1, i+1]],
 * conjugated when w_eff < 0 (K(q, -w) = conj K(q, w)).  No per-visibility
 * taps are stored: the "kernel" buffer holds the lattice instead, as complex64
 * pairs (T[j, i], T[j+1, i]) for j = 0 .. floor(max|w_eff| / dw) and i up to
 * the largest tap distance of a support at |w| = (j + 1) dw.  Supports, the
 * tile work lists and every other part of the operator are those of the exact
 * mode.  Only with precision WSP_FP32_FP64PHASE.  The interpolation error with
 * the default steps is about 1e-4 of the kernel peak on 25-degree fields
 * (bilinear error ~ dq^2/8 max|d2K/dq2| + dw^2/8 max|d2K/dw2|). */

/* Tap layouts (exact mode).  The taps of every visibility are cut by the 64 x
 * 64 grid tiles they fall in and by bands of band_rows tile rows; a "run" is
 * the part of one visibility's footprint in one band of one tile, row-major.
 * The kernel buffer holds the tile work items one after the other, and an
 * item its bands in turn.  Within a band:
 *   WSP_LAYOUT_RUNS: the runs one after the other, each contiguous;
 *   WSP_LAYOUT_INTERLEAVED: the runs sorted by length (longest first), in
 *     groups of 64; a group stores tap 0 of each of its runs, then tap 1 of
 *     each run still that long, and so on, so that one wavefront reads a
 *     group with one lane per run and contiguous loads.
 * The interleaved layout makes degrid faster on short runs (no lane looks for
 * the run its tap belongs to) but its grid adds with LDS atomics, and runs of
 * a step collide on cells, which makes it slow; WSP_LAYOUT_AUTO takes
 * contiguous runs.  The layout changes where taps are stored, not their
 * values; results differ only in rounding order.  wsp_kernel_values reads
 * any layout. */

typedef struct wsp_ctx wsp_ctx;

/* Fill *p with defaults: alpha 2, J 4, beta 2.34 J, f 1, K 1, no fold,
 * tolerances 1e-6, 1024 panels, max support 1024, FP32+FP64 phase, k-means
 * tolerance 1e-3 and 100 iterations, device 0.  n and fov_rad are left 0. */
void wsp_default_params(wsp_params *p);

/* Validate *p and create a context on p->device.  F and F^dagger of the K
 * stacks run as G-point transforms along v and u, G = alpha N: for G a power
 * of two from 64 to 8192 with N <= G / 2 (and the transform's workgroup
 * within the device's LDS), as LDS-resident transforms whose twiddle table
 * is uploaded here; otherwise as batched 1-D library FFT plans made here.
 * Their work area lives in the caller's scratch.
 * Errors: WSP_EINVAL (parameters), WSP_EHIP. */
wsp_status wsp_create(const wsp_params *p, wsp_ctx **out);

/* Attach M visibilities.  uvw: device float64 [M][3] (wavelengths); weights:
 * device float64 [M] or NULL (all ones).  Both are copied.  Runs, on the
 * stream, folding (Eq. (8)), the k-means w-stacking of Algorithm 1, the
 * support rule, the sort by (stack, grid tile) and the tile work lists, and
 * returns when they are complete.  Support rule (the paper only says supports
 * shrink with |w - wbar|, Sec. 3.1): J_p = J + 2 ceil(|w_p - wbar_k| s f),
 * s = rho_c / (n_c du), rho_c = fov sqrt(1/2), n_c = sqrt(1 - rho_c^2),
 * du = 1 / (alpha fov).  Any previous binding is dropped.
 * Errors: WSP_EINVAL (M <= 0, non-finite uvw), WSP_ESUPPORT, WSP_EHIP. */
wsp_status wsp_set_uvw(wsp_ctx *ctx, const double *uvw, int64_t m,
                       const double *weights, void *stream);

/* Replace the stack assignment (host arrays: labels int32 [M] in caller order,
 * values in [0, K); centres float64 [K]) and re-plan.  Lets two
 * implementations share one assignment where Algorithm 1 has ties.  Any
 * previous binding is dropped.  Errors: WSP_ESTATE, WSP_EINVAL, WSP_ESUPPORT. */
wsp_status wsp_set_stacks(wsp_ctx *ctx, const int32_t *labels, const double *centres,
                          void *stream);

/* DDE kernels (dde_support = J_D >= 3): d_u, d_v are device complex [M][J_D]
 * (complex64 or complex128 by precision) in the caller's order; both are
 * copied.  Required before wsp_build_kernels when J_D >= 3; kept across
 * wsp_set_stacks, dropped by wsp_set_uvw.  Errors: WSP_ESTATE (no
 * visibilities yet, or dde_support < 3), WSP_EINVAL, WSP_EHIP. */
wsp_status wsp_set_dde(wsp_ctx *ctx, const void *d_u, const void *d_v, void *stream);

/* Copy out the stack assignment (host: labels [M] in caller order or NULL,
 * centres [K]) and the number of k-means iterations run (0 after
 * wsp_set_stacks).  Errors: WSP_ESTATE. */
wsp_status wsp_get_stacks(const wsp_ctx *ctx, int32_t *labels, double *centres,
                          int32_t *iterations);

/* Copy out per-visibility supports J_p (host int32 [M], caller order) and the
 * fold flags (host uint8 [M] or NULL).  Errors: WSP_ESTATE. */
wsp_status wsp_get_support(const wsp_ctx *ctx, int32_t *jp, uint8_t *folded);

/* Statistics of the plan made by wsp_set_uvw / wsp_set_stacks (Sec. 3.1-3.3:
 * the supports of Eq. (5), the w-stacks of Algorithm 1, the tile work lists)
 * and the device memory the library holds itself. */
typedef struct wsp_plan_info {
    int64_t visibilities;     /* M                                                       */
    int64_t taps;             /* sum_p J_p^2                                             */
    int64_t entries;          /* (visibility, 64 x 64 grid tile) overlaps                */
    int64_t runs;             /* (entry, band of band_rows tile rows) parts; 0 in w-plane mode */
    int64_t items;            /* tile work items                                          */
    int64_t tiles;            /* distinct (stack, tile) pairs that hold taps             */
    int64_t split_tiles;      /* tiles whose entries are split over several items       */
    int64_t touched_cells;    /* distinct (stack, grid cell) pairs some tap falls on     */
    int64_t plan_bytes;       /* device bytes the library holds for the context now (its
                                 plan, the DDE kernels, the stack centres), counted
                                 allocation by allocation                              */
    int64_t plan_peak_bytes;  /* the same at its peak during the last wsp_set_uvw /
                                 wsp_set_stacks (planning temporaries included)        */
    int64_t build_temp_bytes; /* upper bound on the device bytes wsp_build_kernels
                                 allocates beyond plan_bytes and frees before it returns
                                 (admission can add it before building)                */
    int64_t last_build_temp_bytes; /* the same, measured during the last build (0 before
                                 one; wsp_build_kernels_noalloc allocates nothing)     */
    int32_t max_support;      /* largest J_p                                              */
    int32_t kmeans_iterations;/* Algorithm 1 iterations (0 after wsp_set_stacks)          */
    int32_t band_rows;        /* tile rows per band of the exact tap layout (0 in w-plane mode) */
    int32_t tap_layout;       /* WSP_LAYOUT_RUNS or WSP_LAYOUT_INTERLEAVED (0 in w-plane mode) */
    int64_t group_steps;      /* interleaved layout: sum over groups of their longest run
                                 (taps / (64 group_steps) is the share of busy lanes) */
    int64_t classes;          /* contiguous runs: classes of neighbouring runs of one shape
                                 (same width, rows and first cell) within a band   */
    int64_t long_taps;        /* taps in classes whose shape has more than 64 taps (when
                                 more than half the taps, grid streams runs instead
                                 of accumulating classes in registers)              */
    int32_t fft_lds;          /* 1: F and F^dagger run as LDS-resident transforms fused
                                 with the image-side steps (G a power of two in
                                 [64, 8192]); 0: batched library passes             */
    int32_t fft_rows;         /* grid rows per stack that F fills and F^dagger reads
                                 (the rows holding work items, or G)                */
} wsp_plan_info;

/* Fill *info.  touched_cells is counted on the device (synchronises it).
 * Errors: WSP_ESTATE (no plan), WSP_EINVAL, WSP_EHIP. */
wsp_status wsp_plan_stats(wsp_ctx *ctx, wsp_plan_info *info);

/* Exact byte sizes of the caller-owned buffers after wsp_set_uvw (the
 * memory the library allocates itself is reported by wsp_plan_stats:
 * plan_bytes held, plus up to build_temp_bytes during a build):
 * kernel taps (sum_p J_p^2 complex values; in w-plane mode the w-plane
 * lattice instead, 16 bytes per sample pair), the K Fourier grids (K G^2
 * complex values) and scratch (FFT work area, M complex values, one complex
 * partial sum per (visibility, grid tile) overlap, and one 64 x 64 complex
 * partial tile per work item of a grid tile split over several items).
 * Errors: WSP_ESTATE. */
wsp_status wsp_footprint(const wsp_ctx *ctx, size_t *kernel_bytes,
                         size_t *grid_bytes, size_t *scratch_bytes);

/* Attach caller-owned device buffers (256-byte aligned) of at least the
 * footprint sizes.  The library only uses them.  Errors: WSP_ESTATE,
 * WSP_ENOMEM_BINDING (NULL or too small), WSP_EINVAL (misaligned). */
wsp_status wsp_bind_memory(wsp_ctx *ctx, void *kernels, size_t kernel_bytes,
                           void *grids, size_t grid_bytes,
                           void *scratch, size_t scratch_bytes);

/* Build every visibility's J_p x J_p taps (Eq. (5) and (6)):
 *   K_p[row, col] = 2 pi int_0^{alpha/2} g(r) exp(-2 pi i w_eff (n(r) - 1))
 *                   J0(2 pi r q) r dr,
 * q = |(u_p, v_p)/du - (U0 + col, V0 + row)|, U0 = floor(u_p/du) - J_p/2 + 1,
 * g = 2-D Fourier transform of the radial KB blob, by adaptive Gauss-Kronrod
 * (7, 15) quadrature with the tolerances of the parameters.  Blocks until
 * complete.  Returns WSP_WARN_QUAD_MAXEVAL if a visibility reached
 * quad_max_panels.  In w-plane mode it integrates the lattice of w-planes
 * with the same quadrature and tolerances instead.
 * Errors: WSP_ESTATE, WSP_ENOMEM_BINDING, WSP_EHIP. */
wsp_status wsp_build_kernels(wsp_ctx *ctx, void *stream);

/* The same build for the visibilities first .. first+count-1 of the build
 * order (costliest first), so a caller can report progress on long builds.
 * Parts must follow each other from first = 0; the operator is usable once
 * all M are built.  In w-plane mode the part starting at 0 builds the whole
 * lattice and later parts only advance the count.  Errors: as
 * wsp_build_kernels, WSP_EINVAL (range), WSP_ESTATE (out of order). */
wsp_status wsp_build_kernels_part(wsp_ctx *ctx, int64_t first, int64_t count, void *stream);

/* wsp_build_kernels for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same taps, bit for bit, but the build
 * temporaries (quadrature partitions, radial samples, scan storage) live in
 * a static device array of 64 MiB that each GPU using the library holds until
 * the process ends, instead of memory the build allocates.  Visibilities are
 * processed in batches sized so that the worst case of a batch fits.  The
 * call allocates nothing; the kernel taps still go to the caller's bound
 * buffer.  Every call on one GPU shares that GPU's array: calls that overlap
 * in time on one GPU (other contexts or threads) race and must be serialised
 * by the caller.  Blocks until complete.  Errors: as wsp_build_kernels, and
 * WSP_ENOMEM_BINDING if one visibility's temporaries exceed the array. */
wsp_status wsp_build_kernels_noalloc(wsp_ctx *ctx, void *stream);

/* Quadrature statistics of the last build: total panels, and visibilities
 * whose quadrature could not meet the tolerance (the panel cap was reached,
 * or a panel over the tolerance was too narrow to split).  Errors: WSP_ESTATE. */
wsp_status wsp_quad_stats(const wsp_ctx *ctx, int64_t *panels, int64_t *capped);

/* y = Phi x (Eq. (2)-(5)): per stack, taper and w-bar chirp (S~_k), zero pad
 * (Z), forward FFT (F), then the sparse convolution with the built taps (GC_k)
 * and the weights (W_k); folded visibilities are conjugated (Eq. (8)).
 * image: device real [N][N]; vis: device complex [M] (caller order),
 * overwritten.  Asynchronous on the stream.  Errors: WSP_ESTATE, WSP_EINVAL,
 * WSP_EHIP. */
wsp_status wsp_degrid(wsp_ctx *ctx, const void *image, void *vis, void *stream);

/* image = Re Phi^dagger vis (Eq. (7)): gridding with the conjugated taps,
 * inverse FFT, crop, conjugate stack correction, real part, summed over
 * stacks.  vis: device complex [M] (caller order); image: device real [N][N],
 * overwritten.  Asynchronous on the stream.  Errors as wsp_degrid. */
wsp_status wsp_grid(wsp_ctx *ctx, const void *vis, void *image, void *stream);

/* wsp_degrid / wsp_grid on the caller's (grids, scratch) pair instead of
 * the bound one (each at least its wsp_footprint size, 256-byte aligned,
 * device memory the caller owns).  The taps stay the bound ones.  Several
 * requests on one context can then run at once on different streams, each
 * with its own pair (the serving loop's slots).  Host calls on one context
 * must still not overlap.  Errors: as wsp_degrid, WSP_ENOMEM_BINDING (a
 * buffer NULL or too small), WSP_EINVAL (misaligned). */
wsp_status wsp_degrid_ws(wsp_ctx *ctx, const void *image, void *vis, void *grids, size_t grid_bytes,
                         void *scratch, size_t scratch_bytes, void *stream);
wsp_status wsp_grid_ws(wsp_ctx *ctx, const void *vis, void *image, void *grids, size_t grid_bytes,
                       void *scratch, size_t scratch_bytes, void *stream);

/* Linear polarisation (Sec. 3.3, Eq. (9)).  Stokes Q and U are real images,
 * P = Q + iU and y_P = y_Q + i y_U.  Folding reflects each real Stokes image's
 * visibilities on its own: for a folded visibility (w < 0 given)
 *     y_P(u, v, w) = conj( y_Q(-u, -v, -w) - i y_U(-u, -v, -w) ),
 * not the conjugate of y_P itself.  wsp_degrid_pol: vis = Phi Q + i Phi U,
 * each Phi with its Eq. (8) conjugation.  q_image, u_image: device real [N][N];
 * vis: device complex [M] (caller order), overwritten.  Runs the degrid
 * pipeline twice; vis must not alias an image.  Asynchronous on the stream.
 * Errors as wsp_degrid. */
wsp_status wsp_degrid_pol(wsp_ctx *ctx, const void *q_image, const void *u_image, void *vis,
                          void *stream);

/* Adjoint of wsp_degrid_pol under the real inner product:
 *     q_image = Re Phi^dagger vis,   u_image = Re Phi^dagger (-i vis),
 * each overwritten (device real [N][N], distinct).  Asynchronous on the
 * stream.  Errors as wsp_grid, WSP_EINVAL if the two images are the same buffer. */
wsp_status wsp_grid_pol(wsp_ctx *ctx, const void *vis, void *q_image, void *u_image, void *stream);

/* Test hook: copy the taps of visibility p (caller order) to host memory
 * (complex, J_p^2 values, row-major [row][col], rows along v) and return J_p
 * and the unwrapped base indices U0, V0.  out may be NULL to query J_p only.
 * In w-plane mode the taps are interpolated from the lattice as degrid and
 * grid do.  Synchronises the device.  Errors: WSP_ESTATE, WSP_EINVAL, WSP_EHIP. */
wsp_status wsp_kernel_values(wsp_ctx *ctx, int64_t p, void *out, int32_t *jp,
                             int32_t *u0, int32_t *v0);

/* Per-stage timing of wsp_degrid / wsp_grid with HIP events recorded on the
 * call's stream around each launch.  wsp_set_timing(ctx, 1) resets the totals
 * and starts recording, 0 stops.  wsp_stage_times waits for the recorded
 * events and returns the summed milliseconds and launch counts per stage
 * (WSP_NSTAGES entries each, in the order of the WSP_STAGE_* indices).
 * counts may be NULL.  Errors: WSP_EINVAL. */
#define WSP_NSTAGES 7
#define WSP_STAGE_TAPER_PAD 0     /* S~_k and Z                      */
#define WSP_STAGE_FFT_FORWARD 1   /* F, all stacks                   */
#define WSP_STAGE_DEGRID 2        /* GC_k and W_k                    */
#define WSP_STAGE_ZERO 3          /* clearing the grids              */
#define WSP_STAGE_GRID 4          /* W_k and GC_k^dagger             */
#define WSP_STAGE_FFT_INVERSE 5   /* F^dagger, all stacks            */
#define WSP_STAGE_CROP_UNTAPER 6  /* Z^dagger, S~_k^dagger, Re, sum  */
wsp_status wsp_set_timing(wsp_ctx *ctx, int32_t enable);
wsp_status wsp_stage_times(wsp_ctx *ctx, double *ms, int64_t *counts);

/* Free the library-owned plan and FFT plan.  Does not touch bound buffers. */
void wsp_destroy(wsp_ctx *ctx);

/* Thread-local description of the last non-zero status. */
const char *wsp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WSP_H */
