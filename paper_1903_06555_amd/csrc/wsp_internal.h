// Internal declarations shared by the host API and the HIP kernels of libwsp.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "wsp.h"

namespace wsp {

// Device memory the library allocates for a context (its plan, copies, and
// the temporaries of planning and building), tracked so that the footprint
// it reports is exact.  Every allocation of a context's calls goes through
// dmalloc / dfree while that context's tracker is current on the thread
// (TrackScope, set by each entry point).
struct AllocTrack {
    size_t cur = 0;   // bytes live now
    size_t peak = 0;  // high-water mark since the last reset
    std::unordered_map<void *, size_t> live;
};
extern thread_local AllocTrack *g_track;

inline hipError_t dmalloc(void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess && g_track && *p) {
        g_track->live[*p] = bytes;
        g_track->cur += bytes;
        if (g_track->cur > g_track->peak) g_track->peak = g_track->cur;
    }
    return e;
}
template <typename T>
inline hipError_t dmalloc(T **p, size_t bytes) {
    return dmalloc(reinterpret_cast<void **>(p), bytes);
}
// Frees are best effort (release paths have no caller to report to).
inline void dfree(void *p) {
    if (g_track && p) {
        auto it = g_track->live.find(p);
        if (it != g_track->live.end()) {
            g_track->cur -= it->second;
            g_track->live.erase(it);
        }
    }
    (void)hipFree(p);
}

struct TrackScope {
    AllocTrack *prev;
    explicit TrackScope(AllocTrack *t) : prev(g_track) { g_track = t; }
    ~TrackScope() { g_track = prev; }
};

constexpr int kWave = 64;
constexpr int kTile = 64;          // grid tile side (cells) used for sort keys
constexpr int kMaxPanels = 1024;   // quadrature panels per visibility (LDS bound)
constexpr int kProbes = 8;         // probe distances used by the panel error estimate
constexpr int64_t kItemTaps = 1 << 19; // default taps per tile work item (bound before the last entry)
// tile rows per band of the band-major tap layout: 8 or 16, chosen per plan
// (16 when entries are small, so that a run is most of its entry)
constexpr int kMaxBandRows = 16;

// Geometry of one operator, all derived once on the host (FP64).
struct Geom {
    int n;               // image side N
    int G;               // grid side alpha N
    int J;               // KB support
    int n_stacks;        // K
    int taper_terms;     // terms of the FP64 series of g
    double fov;          // radians
    double alpha;
    double inv_du;       // alpha fov: wavelengths -> grid cells
    double du;           // 1 / (alpha fov)
    double dl;           // fov / N
    double r_max;        // alpha / 2 (cycles per cell)
    double beta;         // KB shape
    double a;            // J / 2
    double taper_norm;   // 2 pi a^2 / I0(beta)
    double slope;        // support slope s f (cells per wavelength of |w - wbar|)
    // grid rows that hold work items: [0, rows_lo) and [G - rows_hi, G) of
    // every stack (rows_lo = G, rows_hi = 0 when the pruning does not pay)
    int rows_lo;
    int rows_hi;
    // w-plane mode (kernels interpolated from the lattice K(i dq, j dw))
    bool planes;
    double plane_dq, plane_inv_dq;
    double plane_dw, plane_inv_dw;
    // DDE convolution (Eq. (11)): half width h of the per-visibility kernel D
    int dde_h;
    int64_t item_taps;   // taps per tile work item (before its last entry)
    int band_rows_param; // requested band height (0: chosen from the plan)
    int tap_layout_param; // requested tap layout (WSP_LAYOUT_*)
};

__host__ __device__ inline bool row_used(int V, const Geom &g) {
    return V < g.rows_lo || V >= g.G - g.rows_hi;
}

// Tap layout.  A visibility's J_p x J_p taps occupy one contiguous block
// (at tap_off[p]).  Inside it the taps are grouped by the 64 x 64 grid tile
// they fall in (tiles of the wrapped footprint starting at (u0w, v0w)):
// sub-blocks follow each other tile row by tile row, and each sub-block is
// row-major.  A work item therefore streams each of its entries as one
// contiguous run.
__host__ __device__ inline int64_t blocked_entry_offset(int r0, int nr, int c0, int jp) {
    return (int64_t)r0 * jp + (int64_t)nr * c0;
}

__host__ __device__ inline int64_t blocked_tap_index(int row, int col, int jp, int u0w, int v0w) {
    const int tvy = (v0w + row) / kTile, tvx = (u0w + col) / kTile;
    int r0 = tvy * kTile - v0w;
    r0 = r0 < 0 ? 0 : r0;
    int r1 = (tvy + 1) * kTile - v0w;
    r1 = r1 > jp ? jp : r1;
    int c0 = tvx * kTile - u0w;
    c0 = c0 < 0 ? 0 : c0;
    int c1 = (tvx + 1) * kTile - u0w;
    c1 = c1 > jp ? jp : c1;
    return blocked_entry_offset(r0, r1 - r0, c0, jp) + (int64_t)(row - r0) * (c1 - c0) + (col - c0);
}

// Library-owned, per-visibility plan.  "Caller" arrays are in the caller's
// order; the others are in sorted (stack, tile) order.
struct Plan {
    int64_t m = 0;
    // caller order
    double *u = nullptr, *v = nullptr, *w = nullptr;   // folded coordinates
    double *wt_in = nullptr;                            // weights (ones if none given)
    uint8_t *flag = nullptr;                            // folded
    int32_t *label = nullptr;                           // stack
    // sorted order
    int32_t *perm = nullptr;      // sorted -> caller index
    int32_t *iperm = nullptr;     // caller -> sorted index
    double *ux = nullptr;         // u/du - U0 (offset of the visibility from its first tap)
    double *vx = nullptr;
    double *weff = nullptr;       // w - wbar_k
    double *wt = nullptr;         // weight
    int32_t *jp = nullptr;        // support
    int32_t *u0w = nullptr;       // first tap column, wrapped into [0, G)
    int32_t *v0w = nullptr;
    int32_t *stack = nullptr;
    uint8_t *sflag = nullptr;
    int64_t *tap_off = nullptr;   // [m + 1] prefix of jp^2
    int32_t *border = nullptr;    // build order: sorted indices, costliest first
    unsigned long long *stats = nullptr;  // [0] panels, [1] capped visibilities
    int64_t total_taps = 0;
    int32_t max_jp = 0;
    // tile work lists: one entry per (visibility, grid tile) overlap, sorted by
    // (stack, tile) and cut into work items of bounded tap count
    int64_t n_entries = 0;
    int n_items = 0;
    int4 *ent = nullptr;          // [n_entries] {vis, c0 | r0 << 16, nc | nr << 8 | lx0 << 16 | ly0 << 24, key}
    int64_t *ent_off = nullptr;   // [m + 1] first entry of each sorted visibility
    int32_t *ent_sorted = nullptr;// [n_entries] entry indices in (stack, tile) order
    int4 *wrec = nullptr;         // [n_entries] in (stack, tile) order: {index of the entry's first
                                  // tap in the tap array (low, high 32 bits), nc | nr << 8 |
                                  // lx0 << 16 | ly0 << 24, visibility}
    int32_t *item_start = nullptr;// [n_items + 1] ranges of ent_sorted
    uint32_t *item_key = nullptr; // [n_items] (stack, tile) key of each item
    uint8_t *item_sole = nullptr; // [n_items] 1 if the item is its tile's only item
    int32_t *item_slot = nullptr; // [n_items] partial-tile slot of a shared tile's item
    int n_multi = 0;              // items whose tile is split over several items
    int n_mtiles = 0;             // tiles split over several items
    int32_t *itile = nullptr;     // [n_items] items grouped by tile (stable): a tile's items need
                                  // not be adjacent in the work order
    int32_t *mt_first = nullptr;  // [n_mtiles + 1] first position in itile of each split tile (+ n_items)
    int tile_bits = 0;
    // w-plane mode.  Pair row j (j < n_pairs) holds float4 (T[j, i], T[j+1, i])
    // for i < plane_off[j + 1] - plane_off[j]; a visibility with
    // j dw <= |w_eff| < (j + 1) dw reads row j.
    int n_pairs = 0;
    int band_rows = 0;            // pair rows per band of the work order (see make_entries)
    int64_t table_len = 0;        // float4 elements of the lattice
    int64_t *plane_off = nullptr; // [n_pairs + 1] device
    int4 *prec = nullptr;         // [n_entries] in work-list order: {first float4 of the pair row,
                                  // last usable i | conj << 31, dx0 bits, dy0 bits}; (dx0, dy0) is
                                  // the visibility's offset from the entry's first tap
    float *ptw = nullptr;         // [n_entries] in work-list order: w weight s of the upper plane
    // Band-major tap layout of the exact kernels.  A run is the part of an
    // entry that lies in one band (tile_band_rows tile rows): its rows in the band,
    // row-major.  The tap array holds the work items one after the other; an
    // item holds its bands in turn, a band (a "unit", item * bands + band)
    // holds its runs in work-list order.  Runs are numbered twice:
    // "generation" order groups them by visibility (entries in visibility
    // order, bands in order), "layout" order follows the tap array.
    int tile_band_rows = 8;       // tile rows per band (8 or 16)
    int tile_bands = 8;           // bands per tile, 64 / tile_band_rows
    // Interleaved variant (short runs): a band's runs are sorted by length,
    // longest first, and padded with empty runs to a multiple of 64; each group
    // of 64 stores tap k of its runs (those longer than k) together, k = 0, 1,
    // ..., so tap k of the run in lane i of group G sits at
    // grp_tap[G] + sum_j min(len_j, k) + i.
    bool interleaved = false;
    int layout_param = 0;         // requested layout (WSP_LAYOUT_*)
    int64_t n_runs_padded = 0;    // layout slots (interleaved: multiple of 64 per unit)
    int64_t group_steps = 0;      // sum over groups of their longest run
    int32_t *run_lay = nullptr;   // [n_runs] generation order: layout slot of the run
    uint16_t *len16 = nullptr;    // [n_runs_padded] layout order: run length (0 = padding)
    uint32_t *suf = nullptr;      // [n_runs_padded] layout order: sum of len over the group from here on
    int64_t *grp_tap = nullptr;   // [n_runs_padded / 64 + 1] first tap of each group
    int64_t n_runs = 0;
    int32_t *run_first = nullptr; // [n_entries + 1] first run (generation order) of each entry
    int64_t *run_tap = nullptr;   // [n_runs] generation order: index of the run's first tap
                                  // (contiguous runs only)
    int4 *runrec = nullptr;       // [n_runs_padded] layout order: {first tap of the run (of its
                                  // group, interleaved) relative to its unit, cell0 | nc << 16 |
                                  // nrows << 24, visibility, generation index (-1: padding)}
                                  // (cell0: band-relative tile cell of the run's first tap)
    // Contiguous-runs layout: within a unit, runs of one shape (width, rows,
    // first cell) are neighbours (a class); their taps are consecutive blocks
    // of equal length.
    int64_t n_classes = 0;
    int64_t long_taps = 0;        // taps in classes of more than 64 taps per run
    int4 *clsrec = nullptr;       // [n_classes] {first tap relative to its unit, first run (layout),
                                  // runs, cell0 | nc << 16 | nrows << 24}
    int32_t *unit_cls0 = nullptr; // [n_items * bands + 1] first class of each unit
    int32_t *unit_order = nullptr;// [n_items * bands] units by decreasing taps (ties: by index)
    int32_t *unit_run0 = nullptr; // [n_items * bands + 1] first run (layout order) of each unit
    int64_t *unit_tap0 = nullptr; // [n_items * bands + 1] first tap of each unit
};

// Position in the tap array of tap (row, col) of sorted visibility p (exact
// kernels): its entry is the tile of the wrapped footprint it falls in, its
// run the band of that tile row.
struct TapLayout {
    const int64_t *ent_off;
    const int32_t *run_first;
    const int64_t *run_tap;   // contiguous runs
    const int32_t *run_lay;   // interleaved: slot of each run, and its group's data
    const uint16_t *len16;
    const uint32_t *suf;
    const int64_t *grp_tap;
    int band_rows;
    bool interleaved;
};

inline TapLayout tap_layout(const Plan &pl) {
    return TapLayout{pl.ent_off, pl.run_first, pl.run_tap, pl.run_lay, pl.len16,
                     pl.suf,     pl.grp_tap,   pl.tile_band_rows, pl.interleaved};
}

// Taps stored before tap k of the run in lane i of an interleaved group: the
// runs of the group at least k long (a prefix, lengths descending) hold k
// taps each before step k, the others all theirs, plus the i runs of lanes
// before i at step k.
__device__ __forceinline__ int64_t interleaved_position(const TapLayout &L, int64_t slot, int k) {
    const int64_t g0 = slot & ~(int64_t)63;
    const int lane = (int)(slot & 63);
    int lo = 0, hi = 64;  // t = number of runs with length >= k
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)L.len16[g0 + mid] >= k) lo = mid + 1;
        else hi = mid;
    }
    const int64_t rest = lo < 64 ? (int64_t)L.suf[g0 + lo] : 0;
    return L.grp_tap[g0 >> 6] + (int64_t)k * lo + rest + lane;
}

__device__ __forceinline__ int64_t tap_position(const TapLayout &L, int p, int row, int col, int jp,
                                                int u0w, int v0w) {
    const int tx0 = u0w / kTile, ty0 = v0w / kTile;
    const int tvy = (v0w + row) / kTile, tvx = (u0w + col) / kTile;
    const int ntx = (u0w + jp - 1) / kTile - tx0 + 1;
    const int64_t e = L.ent_off[p] + (int64_t)(tvy - ty0) * ntx + (tvx - tx0);
    int r0 = tvy * kTile - v0w;
    r0 = r0 < 0 ? 0 : r0;
    int c0 = tvx * kTile - u0w;
    c0 = c0 < 0 ? 0 : c0;
    int c1 = (tvx + 1) * kTile - u0w;
    c1 = c1 > jp ? jp : c1;
    const int ly = v0w + row - tvy * kTile;   // tile row of the tap
    const int ly0 = v0w + r0 - tvy * kTile;   // tile row of the entry's first row
    const int br = L.band_rows;
    const int b = ly / br, b0 = ly0 / br;
    const int lo = ly0 > b * br ? ly0 : b * br;  // first tile row of the run
    const int k = (ly - lo) * (c1 - c0) + (col - c0);  // tap of the run
    const int64_t run = L.run_first[e] + (b - b0);
    if (L.interleaved) return interleaved_position(L, L.run_lay[run], k);
    return L.run_tap[run] + k;
}

// Stages timed with HIP events when timing is enabled (wsp_set_timing).
enum Stage { kStTaperPad = 0, kStFftForward, kStDegrid, kStZero, kStGrid, kStFftInverse,
             kStCropUntaper, kNumStages };

struct StageTimer {
    bool enabled = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kNumStages];
    std::vector<hipEvent_t> pool;
    double ms[kNumStages] = {};
    int64_t count[kNumStages] = {};
};

}  // namespace wsp

struct wsp_ctx {
    wsp_params p{};
    wsp::Geom g{};
    int device = 0;
    // F as two passes of batched 1-D transforms of length G: along V over the
    // K x N rows of the half-size buffer (columns of the padded image that hold
    // pixels), and along U over the K x G rows of the grids
    hipfftHandle fft_v = 0, fft_u = 0;
    bool fft_v_made = false, fft_u_made = false;
    // U passes over the used rows only (see Geom::rows_lo): batches of
    // rows_lo, rows_hi + rows_lo (one stack's top band and the next stack's
    // bottom band are adjacent) and rows_hi rows
    hipfftHandle fft_ulo = 0, fft_ujoin = 0, fft_uhi = 0;
    bool fft_ulo_made = false, fft_ujoin_made = false, fft_uhi_made = false;
    size_t fft_work_base = 0;  // work area of fft_v and fft_u
    size_t fft_work = 0;
    // LDS-resident transforms (fft.hip) instead of the library passes, when
    // G is a power of two in [64, 8192] and a transform fits one workgroup's
    // LDS; fft_tw holds the twiddles of their Stockham passes (< G entries)
    bool fft_lds = false;
    void *fft_tw = nullptr;
    // the planned work items' grid tiles: a bitmap (one bit per 64 x 64 tile)
    // and a list of keys (stack | ty | tx); LDS transforms only
    uint64_t *fft_tile_bits = nullptr;
    uint32_t *fft_tile_list = nullptr;
    int n_fft_tiles = 0;
    wsp::Plan plan;
    bool planned = false;
    std::vector<double> centres;   // host copy of the stack centres
    double *plan_centres = nullptr; // device copy
    int iterations = 0;
    void *taps = nullptr;
    size_t taps_bytes = 0;
    void *grids = nullptr;
    size_t grid_bytes = 0;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    void *scratch_half = nullptr;   // transform buffers: [K][N][G] (library passes) or the LDS transforms' (inside scratch)
    void *scratch_yw = nullptr;     // weighted adjoint input, sorted order (inside scratch)
    void *scratch_part = nullptr;   // partial tiles of shared grid tiles (inside scratch)
    void *scratch_dpart = nullptr;  // degrid partial sums, one per tile entry (inside scratch)
    void *dde_u = nullptr;          // [M][J_D] DDE kernels along u and v, caller order (owned)
    void *dde_v = nullptr;
    bool dde_set = false;
    bool bound = false;
    bool built = false;
    int64_t built_upto = 0;         // visibilities built so far, in build order
    int64_t quad_panels = 0;
    int64_t quad_capped = 0;
    void *static_scratch = nullptr; // device address of this device's static build workspace
    wsp::AllocTrack track;          // device memory the library holds for this context
    size_t plan_peak = 0;           // peak of track.cur during the last planning call
    size_t build_peak = 0;          // peak above the resident bytes during the last build
    wsp::StageTimer timer;
};

namespace wsp {

size_t cplx_bytes(const wsp_ctx *c);

// plan.hip
hipError_t launch_fold(const double *uvw, const double *wts, int64_t m, int fold,
                       Plan &pl, int *d_bad, hipStream_t s);
hipError_t minmax_w(const Plan &pl, double *wmin, double *wmax, hipStream_t s);
hipError_t kmeans_iteration(const Plan &pl, const double *d_centres, int K,
                            double *h_new_centres, hipStream_t s);
hipError_t make_plan(wsp_ctx *c, const double *d_centres, hipStream_t s, int *support_err);
void free_sorted_plan(Plan &pl);

hipError_t plane_setup(wsp_ctx *c, hipStream_t s);
hipError_t count_touched_cells(const wsp_ctx *c, int64_t *cells);  // synchronous
hipError_t find_sorted_index(const wsp_ctx *c, int64_t p, int64_t *sidx);  // synchronous

// build.hip.  ws == nullptr: the build allocates its temporaries; otherwise
// they are carved from [ws, ws + ws_bytes) and nothing is allocated.
hipError_t launch_build(wsp_ctx *c, int64_t first, int64_t count, hipStream_t s, void *ws = nullptr,
                        size_t ws_bytes = 0);
hipError_t launch_plane_build(wsp_ctx *c, hipStream_t s, void *ws = nullptr, size_t ws_bytes = 0);
size_t build_temp_bytes(const wsp_ctx *c);  // peak temporaries of the allocating build
int build_batch_in(const wsp_ctx *c, size_t cap);  // batch size whose temporaries fit cap (0: none)
// the static build workspace of the current device (see build.hip)
hipError_t static_scratch_init(int device, void **ptr);
size_t static_scratch_bytes();

// api.cpp: stage timing around one launch (no-ops when timing is off)
hipEvent_t stage_begin(wsp_ctx *c, hipStream_t s);
// LDS-resident F and F^dagger with the image-side steps fused (fft.hip); the
// forward and the U passes take a range of stacks [k0, k1)
bool fft_lds_fits(int G, int n, bool fp64, int device);
hipError_t fft_lds_twiddles(int G, bool fp64, void *dev);
size_t fft_lds_scratch_bytes(const Geom &g, bool fp64);
template <bool kFP64>
hipError_t fft_lds_image_in(const Geom &g, const void *image, void *scratch, hipStream_t s);
template <bool kFP64>
hipError_t fft_lds_forward(const Geom &g, void *grids, void *scratch, const void *tw, const uint64_t *tiles,
                           const double *centres, int k0, int k1, hipStream_t s);
template <bool kFP64>
hipError_t fft_lds_inverse(const Geom &g, const void *grids, void *scratch, const void *tw, const uint64_t *tiles,
                           int k0, int k1, hipStream_t s);

template <bool kFP64>
hipError_t fft_lds_zero_tiles(const Geom &g, void *grids, const uint32_t *list, int n_tiles, int tile_bits,
                              hipStream_t s);
void fft_lds_tile_sets(const Geom &g, const std::vector<uint32_t> &keys, int tile_bits, std::vector<uint64_t> *bits,
                       std::vector<uint32_t> *list);
template <bool kFP64>
hipError_t fft_lds_image_out(const Geom &g, void *image, void *scratch, const void *tw, const double *centres,
                             hipStream_t s);
void stage_end(wsp_ctx *c, int stage, hipEvent_t start, hipStream_t s);

// apply.hip
// add_i = 1: vis += i Phi image (instead of vis = Phi image); rot = 1: image =
// Re Phi^dagger (-i vis).  These are the Stokes U halves of Eq. (9).
hipError_t run_degrid(wsp_ctx *c, const void *image, void *vis, hipStream_t s, int add_i = 0);
hipError_t run_grid(wsp_ctx *c, const void *vis, void *image, hipStream_t s, int rot = 0);
hipError_t run_plane_taps(wsp_ctx *c, int64_t sidx, void *out_dev, hipStream_t s);
hipError_t run_exact_taps(wsp_ctx *c, int64_t sidx, void *out_dev, hipStream_t s);

}  // namespace wsp
