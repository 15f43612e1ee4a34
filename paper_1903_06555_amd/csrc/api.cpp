// Host side of the C ABI declared in include/wsp.h: parameter validation,
// the k-means loop of Algorithm 1, buffer binding and the launch sequence.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "wsp_internal.h"

using namespace wsp;

namespace wsp {
thread_local AllocTrack *g_track = nullptr;
}  // namespace wsp

namespace {

thread_local std::string g_err;

wsp_status fail(wsp_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

wsp_status hip_fail(hipError_t e, const char *where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return WSP_EHIP;
}

#define HIP_OR_FAIL(expr, where)                      \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

double bessel_i0(double x) {
    // I0(x) = sum_k (x^2/4)^k / (k!)^2
    double y = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 400; ++k) {
        term *= y / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

void free_caller(Plan &pl) {
    dfree(pl.u);
    dfree(pl.v);
    dfree(pl.w);
    dfree(pl.wt_in);
    dfree(pl.flag);
    dfree(pl.label);
    pl.u = pl.v = pl.w = pl.wt_in = nullptr;
    pl.flag = nullptr;
    pl.label = nullptr;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void destroy_row_plans(wsp_ctx *c) {
    if (c->fft_ulo_made) hipfftDestroy(c->fft_ulo);
    if (c->fft_ujoin_made) hipfftDestroy(c->fft_ujoin);
    if (c->fft_uhi_made) hipfftDestroy(c->fft_uhi);
    c->fft_ulo_made = c->fft_ujoin_made = c->fft_uhi_made = false;
    dfree(c->fft_tile_bits);
    dfree(c->fft_tile_list);
    c->fft_tile_bits = nullptr;
    c->fft_tile_list = nullptr;
    c->n_fft_tiles = 0;
    c->fft_work = c->fft_work_base;
    c->g.rows_lo = c->g.G;
    c->g.rows_hi = 0;
}

// The grid rows that hold work items (tile rows of the item keys), and
// batched library plans for the U passes over just those rows when they
// leave at least a quarter of the grid out; for the LDS transforms, the used
// rows and the bitmap and list of used tiles instead.
hipfftResult make_row_plans(wsp_ctx *c) {
    destroy_row_plans(c);
    const Plan &pl = c->plan;
    const int G = c->g.G, T = G / kTile, K = c->g.n_stacks;
    if (pl.n_items == 0 && !c->fft_lds) return HIPFFT_SUCCESS;
    std::vector<uint32_t> keys((size_t)pl.n_items);
    if (pl.n_items > 0 && hipMemcpy(keys.data(), pl.item_key, sizeof(uint32_t) * keys.size(),
                                    hipMemcpyDeviceToHost) != hipSuccess)
        return HIPFFT_EXEC_FAILED;
    const uint32_t tmask = (1u << pl.tile_bits) - 1;
    int lo_t = 0, hi_t = 0;
    for (uint32_t key : keys) {
        const int ty = (int)((key >> pl.tile_bits) & tmask);
        if (ty < T / 2) lo_t = ty + 1 > lo_t ? ty + 1 : lo_t;
        else hi_t = T - ty > hi_t ? T - ty : hi_t;
    }
    const int rows_lo = lo_t * kTile, rows_hi = hi_t * kTile;
    if (c->fft_lds) {  // the LDS transforms take the used rows and tiles directly
        std::vector<uint64_t> bits;
        std::vector<uint32_t> list;
        fft_lds_tile_sets(c->g, keys, pl.tile_bits, &bits, &list);
        list.push_back(0u);  // never empty (the count excludes it)
        if (dmalloc(&c->fft_tile_bits, sizeof(uint64_t) * bits.size()) != hipSuccess ||
            dmalloc(&c->fft_tile_list, sizeof(uint32_t) * list.size()) != hipSuccess ||
            hipMemcpy(c->fft_tile_bits, bits.data(), sizeof(uint64_t) * bits.size(), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(c->fft_tile_list, list.data(), sizeof(uint32_t) * list.size(), hipMemcpyHostToDevice) !=
                hipSuccess) {
            destroy_row_plans(c);
            return HIPFFT_ALLOC_FAILED;
        }
        c->n_fft_tiles = (int)list.size() - 1;
        if (rows_lo + rows_hi > 0 && rows_lo + rows_hi < G) {
            c->g.rows_lo = rows_lo;
            c->g.rows_hi = rows_hi;
        }
        return HIPFFT_SUCCESS;
    }
    if (4 * (rows_lo + rows_hi) > 3 * G) return HIPFFT_SUCCESS;  // not worth it
    const hipfftType ty = c->p.precision == WSP_FP64 ? HIPFFT_Z2Z : HIPFFT_C2C;
    int len[1] = {G};
    auto make = [&](hipfftHandle *h, bool *made, int batch) -> hipfftResult {
        if (batch <= 0) return HIPFFT_SUCCESS;
        hipfftResult r = hipfftCreate(h);
        if (r != HIPFFT_SUCCESS) return r;
        *made = true;
        hipfftSetAutoAllocation(*h, 0);
        size_t w = 0;
        r = hipfftMakePlanMany(*h, 1, len, nullptr, 1, G, nullptr, 1, G, ty, batch, &w);
        if (w > c->fft_work) c->fft_work = w;
        return r;
    };
    hipfftResult r = make(&c->fft_ulo, &c->fft_ulo_made, rows_lo);
    if (r == HIPFFT_SUCCESS && K > 1) r = make(&c->fft_ujoin, &c->fft_ujoin_made, rows_lo + rows_hi);
    if (r == HIPFFT_SUCCESS) r = make(&c->fft_uhi, &c->fft_uhi_made, rows_hi);
    if (r != HIPFFT_SUCCESS) {
        destroy_row_plans(c);
        return r;
    }
    c->g.rows_lo = rows_lo;
    c->g.rows_hi = rows_hi;
    return HIPFFT_SUCCESS;
}

wsp_status finish_plan_inner(wsp_ctx *c, hipStream_t s);

// Plan, and record the planning call's device-memory peak.
wsp_status finish_plan(wsp_ctx *c, hipStream_t s) {
    const wsp_status st = finish_plan_inner(c, s);
    c->plan_peak = c->track.peak;
    return st;
}

wsp_status finish_plan_inner(wsp_ctx *c, hipStream_t s) {
    int support_err = 0;
    hipError_t e = make_plan(c, c->plan_centres, s, &support_err);
    if (e != hipSuccess) return hip_fail(e, "planning");
    if (support_err & 1) {
        c->planned = false;
        return fail(WSP_ESUPPORT, "a kernel support J_p exceeds max_support");
    }
    if (support_err & 2) {
        c->planned = false;
        return fail(WSP_EINVAL, "a visibility lies beyond 1e9 grid cells");
    }
    if (c->g.dde_h > 0 &&
        (size_t)(2 * c->g.dde_h + 1) * (size_t)c->plan.max_jp * cplx_bytes(c) > 65536) {
        c->planned = false;
        return fail(WSP_ESUPPORT, "DDE convolution: J_D x max J_p' complex values exceed 64 KiB");
    }
    if (support_err & 4) {
        c->planned = false;
        return fail(WSP_EINVAL, "w-plane lattice above 2^31 sample pairs: raise plane_dq or plane_dw");
    }
    if (c->g.planes) {
        e = plane_setup(c, s);
        if (e != hipSuccess) return hip_fail(e, "w-plane records");
    }
    hipfftResult fr = make_row_plans(c);
    if (fr != HIPFFT_SUCCESS) {
        c->planned = false;
        return fail(WSP_EHIP, "transform set-up for the used grid rows failed (" + std::to_string((int)fr) + ")");
    }
    c->planned = true;
    c->bound = false;
    c->built = false;
    c->built_upto = 0;
    return WSP_OK;
}

}  // namespace

size_t wsp::cplx_bytes(const wsp_ctx *c) { return c->p.precision == WSP_FP64 ? 16 : 8; }

namespace {
// the half-size transform buffer: K x N rows of G cells
size_t half_bytes(const wsp_ctx *c) {
    if (c->fft_lds) return fft_lds_scratch_bytes(c->g, c->p.precision == WSP_FP64);
    return (size_t)c->g.n_stacks * c->g.n * c->g.G * cplx_bytes(c);
}
// degrid partial sums: one per run (exact kernels) or per tile entry (w-plane kernels)
size_t n_partials(const wsp_ctx *c) {
    return (size_t)(c->g.planes ? c->plan.n_entries : c->plan.n_runs);
}
}  // namespace

hipEvent_t wsp::stage_begin(wsp_ctx *c, hipStream_t s) {
    if (!c->timer.enabled) return nullptr;
    hipEvent_t ev = nullptr;
    if (!c->timer.pool.empty()) {
        ev = c->timer.pool.back();
        c->timer.pool.pop_back();
    } else if (hipEventCreate(&ev) != hipSuccess) {
        return nullptr;
    }
    hipEventRecord(ev, s);
    return ev;
}

void wsp::stage_end(wsp_ctx *c, int stage, hipEvent_t start, hipStream_t s) {
    if (!start) return;
    hipEvent_t ev = nullptr;
    if (!c->timer.pool.empty()) {
        ev = c->timer.pool.back();
        c->timer.pool.pop_back();
    } else if (hipEventCreate(&ev) != hipSuccess) {
        c->timer.pool.push_back(start);
        return;
    }
    hipEventRecord(ev, s);
    c->timer.pending[stage].emplace_back(start, ev);
}

namespace {
void drain_timer(wsp_ctx *c) {
    for (int st = 0; st < kNumStages; ++st) {
        for (auto &pr : c->timer.pending[st]) {
            float ms = 0.0f;
            if (hipEventSynchronize(pr.second) == hipSuccess &&
                hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
                c->timer.ms[st] += ms;
                c->timer.count[st] += 1;
            }
            c->timer.pool.push_back(pr.first);
            c->timer.pool.push_back(pr.second);
        }
        c->timer.pending[st].clear();
    }
}
}  // namespace

extern "C" {

void wsp_default_params(wsp_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->oversample = 2.0;
    p->kb_support = 4;
    p->kb_beta = 0.0;
    p->support_scale = 1.0;
    p->n_stacks = 1;
    p->fold_conjugate = 0;
    p->quad_rel_tol = 1e-6;
    p->quad_abs_tol = 1e-6;
    p->quad_max_panels = kMaxPanels;
    p->max_support = 1024;
    p->precision = WSP_FP32_FP64PHASE;
    p->kmeans_tol = 1e-3;
    p->kmeans_max_iter = 100;
    p->device = 0;
}

const char *wsp_last_error(void) { return g_err.c_str(); }

wsp_status wsp_create(const wsp_params *pp, wsp_ctx **out) {
    if (!pp || !out) return fail(WSP_EINVAL, "null argument");
    *out = nullptr;
    const wsp_params &p = *pp;
    if (p.n < 2 || p.n % 2) return fail(WSP_EINVAL, "n must be even and >= 2");
    if (!(p.oversample >= 1.0) || !std::isfinite(p.oversample))
        return fail(WSP_EINVAL, "oversample must be >= 1");
    double gd = p.oversample * p.n;
    long G = std::lround(gd);
    if (std::fabs(gd - (double)G) > 1e-9 || G % kTile || G > (1L << 20))
        return fail(WSP_EINVAL, "oversample * n must be an integer multiple of 64 (<= 2^20)");
    if (!(p.fov_rad > 0.0) || !std::isfinite(p.fov_rad))
        return fail(WSP_EINVAL, "fov_rad must be positive");
    if (!(p.oversample * p.oversample * p.fov_rad / 2.0 < 1.0))
        return fail(WSP_EINVAL, "oversample^2 fov / 2 must be < 1 (kernel integral past the horizon)");
    if (p.kb_support < 2 || p.kb_support % 2 || p.kb_support > 32)
        return fail(WSP_EINVAL, "kb_support must be even in [2, 32]");
    if (!(p.kb_beta >= 0.0) || !std::isfinite(p.kb_beta)) return fail(WSP_EINVAL, "kb_beta must be >= 0");
    if (!(p.support_scale >= 1.0) || !std::isfinite(p.support_scale))
        return fail(WSP_EINVAL, "support_scale must be >= 1");
    if (p.n_stacks < 1 || p.n_stacks > 256) return fail(WSP_EINVAL, "n_stacks must be in [1, 256]");
    if (p.fold_conjugate != 0 && p.fold_conjugate != 1)
        return fail(WSP_EINVAL, "fold_conjugate must be 0 or 1");
    if (!(p.quad_rel_tol >= 0.0) || !(p.quad_abs_tol >= 0.0) ||
        !(p.quad_rel_tol > 0.0 || p.quad_abs_tol > 0.0) || !std::isfinite(p.quad_rel_tol) ||
        !std::isfinite(p.quad_abs_tol))
        return fail(WSP_EINVAL, "quadrature tolerances must be >= 0 and not both 0");
    if (p.quad_max_panels < 8 || p.quad_max_panels > kMaxPanels)
        return fail(WSP_EINVAL, "quad_max_panels must be in [8, 1024]");
    if (p.max_support < p.kb_support || p.max_support > 8192)
        return fail(WSP_EINVAL, "max_support must be in [kb_support, 8192]");
    if (p.precision != WSP_FP32_FP64PHASE && p.precision != WSP_FP64)
        return fail(WSP_EINVAL, "unknown precision");
    if (!(p.kmeans_tol >= 0.0) || p.kmeans_max_iter < 1)
        return fail(WSP_EINVAL, "kmeans_tol must be >= 0 and kmeans_max_iter >= 1");
    if (p.device < 0) return fail(WSP_EINVAL, "device must be >= 0");
    if (p.kernel_mode != WSP_KERNELS_EXACT && p.kernel_mode != WSP_KERNELS_PLANES)
        return fail(WSP_EINVAL, "unknown kernel_mode");
    if (p.kernel_mode == WSP_KERNELS_PLANES && p.precision != WSP_FP32_FP64PHASE)
        return fail(WSP_EINVAL, "w-plane kernels need precision WSP_FP32_FP64PHASE");
    if (p.dde_support < 0 || p.dde_support > 15 || (p.dde_support > 1 && p.dde_support % 2 == 0))
        return fail(WSP_EINVAL, "dde_support must be 0, 1 or odd in [3, 15]");
    if (p.dde_support > 1 && p.kernel_mode == WSP_KERNELS_PLANES)
        return fail(WSP_EINVAL, "DDE convolution needs stored (exact) kernels");
    if (p.item_taps < 0 || p.item_taps > (1 << 24))
        return fail(WSP_EINVAL, "item_taps must be in [0, 2^24] (0 = default)");
    if (p.band_rows != 0 && p.band_rows != 8 && p.band_rows != 16)
        return fail(WSP_EINVAL, "band_rows must be 0, 8 or 16");
    if (p.tap_layout < WSP_LAYOUT_AUTO || p.tap_layout > WSP_LAYOUT_INTERLEAVED)
        return fail(WSP_EINVAL, "tap_layout must be WSP_LAYOUT_AUTO, _RUNS or _INTERLEAVED");
    if (!(p.plane_dq >= 0.0) || !(p.plane_dw >= 0.0) || !std::isfinite(p.plane_dq) ||
        !std::isfinite(p.plane_dw) || p.plane_dq > 1.0)
        return fail(WSP_EINVAL, "plane_dq must be in [0, 1] and plane_dw >= 0 (0 = default)");

    Geom g{};
    g.n = p.n;
    g.G = (int)G;
    g.J = p.kb_support;
    g.n_stacks = p.n_stacks;
    g.fov = p.fov_rad;
    g.alpha = p.oversample;
    g.inv_du = p.oversample * p.fov_rad;
    g.du = 1.0 / (p.oversample * p.fov_rad);
    g.dl = p.fov_rad / p.n;
    g.r_max = 0.5 * p.oversample;
    g.beta = p.kb_beta > 0.0 ? p.kb_beta : 2.34 * p.kb_support;
    g.a = 0.5 * p.kb_support;
    g.taper_norm = 2.0 * M_PI * g.a * g.a / bessel_i0(g.beta);
    double rho_c = p.fov_rad * std::sqrt(0.5);
    double n_c = std::sqrt(1.0 - rho_c * rho_c);
    g.slope = (rho_c / (n_c * g.du)) * p.support_scale;
    g.rows_lo = g.G;  // all grid rows, until a plan narrows them
    g.rows_hi = 0;
    g.planes = p.kernel_mode == WSP_KERNELS_PLANES;
    g.plane_dq = p.plane_dq > 0.0 ? p.plane_dq : 1.0 / 64.0;
    g.plane_dw = p.plane_dw > 0.0 ? p.plane_dw : 1.0 / 16.0;
    g.plane_inv_dq = 1.0 / g.plane_dq;
    g.plane_inv_dw = 1.0 / g.plane_dw;
    g.dde_h = p.dde_support > 1 ? (p.dde_support - 1) / 2 : 0;
    g.item_taps = p.item_taps > 0 ? (int64_t)p.item_taps : kItemTaps;
    g.band_rows_param = p.band_rows;
    g.tap_layout_param = p.tap_layout;
    double xr = 2.0 * M_PI * g.a * g.r_max;
    double ymax = std::fmax(0.25 * g.beta * g.beta, std::fabs(0.25 * (g.beta * g.beta - xr * xr)));
    int terms = (int)std::ceil(2.0 * std::sqrt(ymax)) + 30;
    if (terms > 128) return fail(WSP_EINVAL, "kb_beta too large for the taper series");
    g.taper_terms = terms;

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (p.device >= ndev) return fail(WSP_EINVAL, "no such device");
    HIP_OR_FAIL(hipSetDevice(p.device), "hipSetDevice");

    // the device address of this device's static build workspace (looked up
    // once per device, with the device current)
    void *static_ws = nullptr;
    HIP_OR_FAIL(static_scratch_init(p.device, &static_ws), "hipGetSymbolAddress (static build workspace)");

    wsp_ctx *c = new (std::nothrow) wsp_ctx();
    if (!c) return fail(WSP_EHIP, "out of host memory");
    c->static_scratch = static_ws;
    TrackScope track(&c->track);
    c->p = p;
    c->g = g;
    c->device = p.device;
    c->fft_lds = fft_lds_fits(g.G, g.n, p.precision == WSP_FP64, p.device);
    if (c->fft_lds) {
        e = dmalloc(&c->fft_tw, (p.precision == WSP_FP64 ? 16 : 8) * (size_t)g.G);
        if (e == hipSuccess) e = fft_lds_twiddles(g.G, p.precision == WSP_FP64, c->fft_tw);
        if (e != hipSuccess) {
            dfree(c->fft_tw);
            delete c;
            return hip_fail(e, "twiddle table");
        }
        c->g.rows_lo = g.G;
        c->g.rows_hi = 0;
    } else {
        const hipfftType ty = p.precision == WSP_FP64 ? HIPFFT_Z2Z : HIPFFT_C2C;
        int len[1] = {g.G};
        size_t wv = 0, wu = 0;
        hipfftResult r = hipfftCreate(&c->fft_v);
        if (r == HIPFFT_SUCCESS) {
            c->fft_v_made = true;
            hipfftSetAutoAllocation(c->fft_v, 0);
            r = hipfftMakePlanMany(c->fft_v, 1, len, nullptr, 1, g.G, nullptr, 1, g.G, ty,
                                   g.n_stacks * g.n, &wv);
        }
        if (r == HIPFFT_SUCCESS) r = hipfftCreate(&c->fft_u);
        if (r == HIPFFT_SUCCESS) {
            c->fft_u_made = true;
            hipfftSetAutoAllocation(c->fft_u, 0);
            r = hipfftMakePlanMany(c->fft_u, 1, len, nullptr, 1, g.G, nullptr, 1, g.G, ty,
                                   g.n_stacks * g.G, &wu);
        }
        if (r != HIPFFT_SUCCESS) {
            if (c->fft_v_made) hipfftDestroy(c->fft_v);
            if (c->fft_u_made) hipfftDestroy(c->fft_u);
            delete c;
            return fail(WSP_EHIP, "hipfftMakePlanMany failed (" + std::to_string((int)r) + ")");
        }
        c->fft_work = wv > wu ? wv : wu;  // the passes run in turn: one work area
        c->fft_work_base = c->fft_work;
        c->g.rows_lo = g.G;
        c->g.rows_hi = 0;
    }
    e = dmalloc(&c->plan_centres, sizeof(double) * g.n_stacks);
    if (e != hipSuccess) {
        if (c->fft_v_made) hipfftDestroy(c->fft_v);
        if (c->fft_u_made) hipfftDestroy(c->fft_u);
        dfree(c->fft_tw);
        delete c;
        return hip_fail(e, "hipMalloc centres");
    }
    *out = c;
    return WSP_OK;
}

wsp_status wsp_set_uvw(wsp_ctx *c, const double *uvw, int64_t m, const double *weights,
                       void *stream) {
    if (!c || !uvw) return fail(WSP_EINVAL, "null argument");
    if (m <= 0 || m > 0x7FFFFFF0LL) return fail(WSP_EINVAL, "m must be in [1, 2^31)");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    TrackScope track(&c->track);
    hipStream_t s = as_stream(stream);
    Plan &pl = c->plan;
    free_sorted_plan(pl);
    free_caller(pl);
    dfree(c->dde_u);
    dfree(c->dde_v);
    c->dde_u = c->dde_v = nullptr;
    c->dde_set = false;
    c->planned = c->bound = c->built = false;
    c->track.peak = c->track.cur;  // planning peak measured from here (finish_plan records it)
    pl.m = m;
    HIP_OR_FAIL(dmalloc(&pl.u, sizeof(double) * m), "hipMalloc");
    HIP_OR_FAIL(dmalloc(&pl.v, sizeof(double) * m), "hipMalloc");
    HIP_OR_FAIL(dmalloc(&pl.w, sizeof(double) * m), "hipMalloc");
    HIP_OR_FAIL(dmalloc(&pl.wt_in, sizeof(double) * m), "hipMalloc");
    HIP_OR_FAIL(dmalloc(&pl.flag, m), "hipMalloc");
    HIP_OR_FAIL(dmalloc(&pl.label, sizeof(int32_t) * m), "hipMalloc");
    int *d_bad = nullptr;
    HIP_OR_FAIL(dmalloc(&d_bad, sizeof(int)), "hipMalloc");
    hipError_t e = hipMemsetAsync(d_bad, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_fold(uvw, weights, m, c->p.fold_conjugate, pl, d_bad, s);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(d_bad);
    if (e != hipSuccess) return hip_fail(e, "fold");
    if (bad) return fail(WSP_EINVAL, "non-finite uvw or weight");

    // Algorithm 1 (k-means w-stacking), convergence read on the host
    double wmin = 0, wmax = 0;
    e = minmax_w(pl, &wmin, &wmax, s);
    if (e != hipSuccess) return hip_fail(e, "w range");
    const int K = c->g.n_stacks;
    std::vector<double> cen(K), nw(K);
    if (K == 1) {
        cen[0] = 0.5 * (wmin + wmax);
    } else {
        double step = (wmax - wmin) / (double)(K - 1);
        for (int q = 0; q < K; ++q) cen[q] = (double)q * step + wmin;
        cen[K - 1] = wmax;
    }
    const double floor_ = 1e-12 * std::fmax(wmax - wmin, 1.0);
    int it = 0;
    for (it = 1; it <= c->p.kmeans_max_iter; ++it) {
        HIP_OR_FAIL(hipMemcpyAsync(c->plan_centres, cen.data(), sizeof(double) * K,
                                   hipMemcpyHostToDevice, s), "centres");
        e = kmeans_iteration(pl, c->plan_centres, K, nw.data(), s);
        if (e != hipSuccess) return hip_fail(e, "k-means");
        double rel = 0.0;
        for (int q = 0; q < K; ++q)
            rel += std::fabs(nw[q] - cen[q]) / std::fmax(std::fabs(nw[q]), floor_);
        rel /= (double)K;
        cen = nw;
        if (rel < c->p.kmeans_tol) break;
    }
    if (it > c->p.kmeans_max_iter) it = c->p.kmeans_max_iter;
    c->iterations = it;
    c->centres = cen;
    HIP_OR_FAIL(hipMemcpyAsync(c->plan_centres, cen.data(), sizeof(double) * K,
                               hipMemcpyHostToDevice, s), "centres");
    return finish_plan(c, s);
}

wsp_status wsp_set_stacks(wsp_ctx *c, const int32_t *labels, const double *centres, void *stream) {
    if (!c || !labels || !centres) return fail(WSP_EINVAL, "null argument");
    if (!c->plan.u) return fail(WSP_ESTATE, "wsp_set_uvw first");
    const int K = c->g.n_stacks;
    for (int64_t i = 0; i < c->plan.m; ++i)
        if (labels[i] < 0 || labels[i] >= K) return fail(WSP_EINVAL, "label out of range");
    for (int q = 0; q < K; ++q)
        if (!std::isfinite(centres[q])) return fail(WSP_EINVAL, "non-finite centre");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    TrackScope track(&c->track);
    c->track.peak = c->track.cur;
    hipStream_t s = as_stream(stream);
    HIP_OR_FAIL(hipMemcpyAsync(c->plan.label, labels, sizeof(int32_t) * c->plan.m,
                               hipMemcpyHostToDevice, s), "labels");
    HIP_OR_FAIL(hipMemcpyAsync(c->plan_centres, centres, sizeof(double) * K,
                               hipMemcpyHostToDevice, s), "centres");
    c->centres.assign(centres, centres + K);
    c->iterations = 0;
    return finish_plan(c, s);
}

wsp_status wsp_set_dde(wsp_ctx *c, const void *d_u, const void *d_v, void *stream) {
    if (!c || !d_u || !d_v) return fail(WSP_EINVAL, "null argument");
    if (!c->plan.u) return fail(WSP_ESTATE, "wsp_set_uvw first");
    if (c->g.dde_h == 0) return fail(WSP_ESTATE, "dde_support is not set (>= 3)");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    TrackScope track(&c->track);
    const size_t bytes = (size_t)c->plan.m * (size_t)(2 * c->g.dde_h + 1) * cplx_bytes(c);
    if (!c->dde_u) HIP_OR_FAIL(dmalloc(&c->dde_u, bytes), "hipMalloc");
    if (!c->dde_v) HIP_OR_FAIL(dmalloc(&c->dde_v, bytes), "hipMalloc");
    hipStream_t s = as_stream(stream);
    HIP_OR_FAIL(hipMemcpyAsync(c->dde_u, d_u, bytes, hipMemcpyDeviceToDevice, s), "DDE copy");
    HIP_OR_FAIL(hipMemcpyAsync(c->dde_v, d_v, bytes, hipMemcpyDeviceToDevice, s), "DDE copy");
    HIP_OR_FAIL(hipStreamSynchronize(s), "DDE copy");
    c->dde_set = true;
    c->built = false;
    c->built_upto = 0;
    return WSP_OK;
}

wsp_status wsp_get_stacks(const wsp_ctx *c, int32_t *labels, double *centres, int32_t *iterations) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "no plan");
    if (labels) {
        HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
        HIP_OR_FAIL(hipMemcpy(labels, c->plan.label, sizeof(int32_t) * c->plan.m,
                              hipMemcpyDeviceToHost), "labels");
    }
    if (centres) std::memcpy(centres, c->centres.data(), sizeof(double) * c->centres.size());
    if (iterations) *iterations = c->iterations;
    return WSP_OK;
}

wsp_status wsp_get_support(const wsp_ctx *c, int32_t *jp, uint8_t *folded) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "no plan");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    const int64_t m = c->plan.m;
    if (jp) {
        std::vector<int32_t> js(m), perm(m);
        HIP_OR_FAIL(hipMemcpy(js.data(), c->plan.jp, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "jp");
        HIP_OR_FAIL(hipMemcpy(perm.data(), c->plan.perm, sizeof(int32_t) * m, hipMemcpyDeviceToHost), "perm");
        for (int64_t i = 0; i < m; ++i) jp[perm[i]] = js[i];
    }
    if (folded) HIP_OR_FAIL(hipMemcpy(folded, c->plan.flag, m, hipMemcpyDeviceToHost), "flags");
    return WSP_OK;
}

wsp_status wsp_plan_stats(wsp_ctx *c, wsp_plan_info *info) {
    if (!c || !info) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    const size_t resident = c->track.cur;  // before the transient bitmap of the cell count
    TrackScope track(&c->track);
    const Plan &pl = c->plan;
    std::memset(info, 0, sizeof(*info));
    info->visibilities = pl.m;
    info->taps = pl.total_taps;
    info->entries = pl.n_entries;
    info->runs = pl.n_runs;
    info->items = pl.n_items;
    info->tiles = pl.n_items - pl.n_multi + pl.n_mtiles;
    info->split_tiles = pl.n_mtiles;
    int64_t cells = 0;
    HIP_OR_FAIL(count_touched_cells(c, &cells), "touched cells");
    info->touched_cells = cells;
    info->plan_bytes = (int64_t)resident;
    info->plan_peak_bytes = (int64_t)c->plan_peak;
    info->build_temp_bytes = (int64_t)build_temp_bytes(c);
    info->last_build_temp_bytes = (int64_t)c->build_peak;
    info->max_support = pl.max_jp;
    info->kmeans_iterations = c->iterations;
    info->band_rows = c->g.planes ? 0 : pl.tile_band_rows;
    info->tap_layout = c->g.planes ? 0 : (pl.interleaved ? WSP_LAYOUT_INTERLEAVED : WSP_LAYOUT_RUNS);
    info->group_steps = pl.interleaved ? pl.group_steps : 0;
    info->classes = pl.n_classes;
    info->long_taps = pl.long_taps;
    info->fft_lds = c->fft_lds ? 1 : 0;
    info->fft_rows = c->g.rows_lo + c->g.rows_hi;
    return WSP_OK;
}

wsp_status wsp_footprint(const wsp_ctx *c, size_t *kernel_bytes, size_t *grid_bytes,
                         size_t *scratch_bytes) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    const size_t cb = cplx_bytes(c);
    if (kernel_bytes)
        *kernel_bytes = c->g.planes ? (size_t)c->plan.table_len * 16 : (size_t)c->plan.total_taps * cb;
    if (grid_bytes) *grid_bytes = (size_t)c->g.G * c->g.G * c->g.n_stacks * cb;
    if (scratch_bytes)
        *scratch_bytes = align256(c->fft_work) + align256(half_bytes(c)) + align256((size_t)c->plan.m * cb) +
                         align256(n_partials(c) * cb) + (size_t)c->plan.n_multi * kTile * kTile * cb;
    return WSP_OK;
}

}  // extern "C"

namespace {
// Point the operator at a (grids, scratch) pair: the scratch's parts and the
// FFT plans' work area.
bool use_workspace(wsp_ctx *c, void *grids, void *scratch) {
    if (c->fft_work > 0) {
        bool ok = hipfftSetWorkArea(c->fft_v, scratch) == HIPFFT_SUCCESS &&
                  hipfftSetWorkArea(c->fft_u, scratch) == HIPFFT_SUCCESS;
        if (c->fft_ulo_made) ok = ok && hipfftSetWorkArea(c->fft_ulo, scratch) == HIPFFT_SUCCESS;
        if (c->fft_ujoin_made) ok = ok && hipfftSetWorkArea(c->fft_ujoin, scratch) == HIPFFT_SUCCESS;
        if (c->fft_uhi_made) ok = ok && hipfftSetWorkArea(c->fft_uhi, scratch) == HIPFFT_SUCCESS;
        if (!ok) return false;
    }
    c->scratch_half = (char *)scratch + align256(c->fft_work);
    c->scratch_yw = (char *)c->scratch_half + align256(half_bytes(c));
    c->scratch_dpart = (char *)c->scratch_yw + align256((size_t)c->plan.m * cplx_bytes(c));
    c->scratch_part = (char *)c->scratch_dpart + align256(n_partials(c) * cplx_bytes(c));
    c->grids = grids;
    c->scratch = scratch;
    return true;
}

// Run one degrid / grid call on another (grids, scratch) pair, then point
// the operator back at the bound pair.  Kernels and FFTs take their buffer
// addresses when they are launched, so the swap does not affect launches
// already on a stream.
template <typename F>
wsp_status with_workspace(wsp_ctx *c, void *grids, size_t grid_bytes, void *scratch, size_t scratch_bytes,
                          const char *what, F &&run) {
    size_t kb = 0, gb = 0, sb = 0;
    wsp_footprint(c, &kb, &gb, &sb);
    if (!grids || (sb > 0 && !scratch)) return fail(WSP_ENOMEM_BINDING, "null workspace");
    if (grid_bytes < gb || scratch_bytes < sb) return fail(WSP_ENOMEM_BINDING, "workspace smaller than wsp_footprint");
    if (((uintptr_t)grids | (uintptr_t)scratch) & 255u) return fail(WSP_EINVAL, "buffers must be 256-byte aligned");
    void *g0 = c->grids, *s0 = c->scratch;
    if (!use_workspace(c, grids, scratch)) {
        use_workspace(c, g0, s0);
        return fail(WSP_EHIP, "hipfftSetWorkArea failed");
    }
    const hipError_t e = run();
    const bool back = use_workspace(c, g0, s0);
    if (e != hipSuccess) return hip_fail(e, what);
    if (!back) return fail(WSP_EHIP, "hipfftSetWorkArea failed");
    return WSP_OK;
}
}  // namespace

extern "C" {

wsp_status wsp_bind_memory(wsp_ctx *c, void *kernels, size_t kernel_bytes, void *grids,
                           size_t grid_bytes, void *scratch, size_t scratch_bytes) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    size_t kb = 0, gb = 0, sb = 0;
    wsp_footprint(c, &kb, &gb, &sb);
    if (!kernels || !grids || (sb > 0 && !scratch))
        return fail(WSP_ENOMEM_BINDING, "null buffer");
    if (kernel_bytes < kb || grid_bytes < gb || scratch_bytes < sb)
        return fail(WSP_ENOMEM_BINDING, "buffer smaller than wsp_footprint");
    if (((uintptr_t)kernels | (uintptr_t)grids | (uintptr_t)scratch) & 255u)
        return fail(WSP_EINVAL, "buffers must be 256-byte aligned");
    if (!use_workspace(c, grids, scratch)) return fail(WSP_EHIP, "hipfftSetWorkArea failed");
    c->taps = kernels;
    c->taps_bytes = kernel_bytes;
    c->grid_bytes = grid_bytes;
    c->scratch_bytes = scratch_bytes;
    c->bound = true;
    c->built = false;
    c->built_upto = 0;
    return WSP_OK;
}

namespace {
// Build parts [first, first + count); ws == nullptr allocates the temporaries.
wsp_status build_part(wsp_ctx *c, int64_t first, int64_t count, void *stream, void *ws, size_t ws_bytes) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    if (!c->bound) return fail(WSP_ENOMEM_BINDING, "wsp_bind_memory first");
    if (first != c->built_upto) return fail(WSP_ESTATE, "parts must be built in order from 0");
    if (c->g.dde_h > 0 && !c->dde_set) return fail(WSP_ESTATE, "wsp_set_dde first");
    if (count <= 0 || first + count > c->plan.m) return fail(WSP_EINVAL, "bad visibility range");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    TrackScope track(&c->track);
    const size_t resident = c->track.cur;
    c->track.peak = resident;
    struct PeakRecord {  // the build's transient peak, on every return path
        wsp_ctx *c;
        size_t base;
        ~PeakRecord() {
            const size_t over = c->track.peak - base;
            if (over > c->build_peak) c->build_peak = over;
        }
    } record{c, resident};
    if (first == 0) c->build_peak = 0;
    hipStream_t s = as_stream(stream);
    if (c->g.planes) {
        // the lattice serves every visibility: built by the first part
        if (first == 0) {
            HIP_OR_FAIL(launch_plane_build(c, s, ws, ws_bytes), "w-plane build");
        } else {
            c->built_upto = first + count;
            c->built = c->built_upto == c->plan.m;
            return WSP_OK;
        }
    } else {
        HIP_OR_FAIL(launch_build(c, first, count, s, ws, ws_bytes), "build");
    }
    unsigned long long st[2] = {0, 0};
    HIP_OR_FAIL(hipMemcpyAsync(st, c->plan.stats, sizeof(st), hipMemcpyDeviceToHost, s), "stats");
    HIP_OR_FAIL(hipStreamSynchronize(s), "build");
    c->quad_panels = (int64_t)st[0];
    c->quad_capped = (int64_t)st[1];
    c->built_upto = first + count;
    c->built = c->built_upto == c->plan.m;
    if (st[1] > 0) {
        g_err = std::to_string(st[1]) + " visibilities did not meet the quadrature tolerance "
                "(quad_max_panels reached, or a panel too narrow to split)";
        return WSP_WARN_QUAD_MAXEVAL;
    }
    return WSP_OK;
}
}  // namespace

wsp_status wsp_build_kernels_part(wsp_ctx *c, int64_t first, int64_t count, void *stream) {
    return build_part(c, first, count, stream, nullptr, 0);
}

wsp_status wsp_build_kernels_noalloc(wsp_ctx *c, void *stream) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    if (!c->static_scratch) return fail(WSP_EHIP, "static build workspace unavailable");
    if (build_batch_in(c, static_scratch_bytes()) < 1)
        return fail(WSP_ENOMEM_BINDING, "the build temporaries of one visibility exceed the " +
                                            std::to_string(static_scratch_bytes() >> 20) +
                                            " MiB static workspace");
    c->built_upto = 0;
    c->built = false;
    return build_part(c, 0, c->plan.m, stream, c->static_scratch, static_scratch_bytes());
}

wsp_status wsp_build_kernels(wsp_ctx *c, void *stream) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "wsp_set_uvw first");
    c->built_upto = 0;
    c->built = false;
    return wsp_build_kernels_part(c, 0, c->plan.m, stream);
}

wsp_status wsp_quad_stats(const wsp_ctx *c, int64_t *panels, int64_t *capped) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "no build yet");
    if (panels) *panels = c->quad_panels;
    if (capped) *capped = c->quad_capped;
    return WSP_OK;
}

wsp_status wsp_degrid(wsp_ctx *c, const void *image, void *vis, void *stream) {
    if (!c || !image || !vis) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    HIP_OR_FAIL(run_degrid(c, image, vis, as_stream(stream)), "degrid");
    return WSP_OK;
}

wsp_status wsp_grid(wsp_ctx *c, const void *vis, void *image, void *stream) {
    if (!c || !image || !vis) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    HIP_OR_FAIL(run_grid(c, vis, image, as_stream(stream)), "grid");
    return WSP_OK;
}

wsp_status wsp_degrid_ws(wsp_ctx *c, const void *image, void *vis, void *grids, size_t grid_bytes,
                         void *scratch, size_t scratch_bytes, void *stream) {
    if (!c || !image || !vis) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    return with_workspace(c, grids, grid_bytes, scratch, scratch_bytes, "degrid",
                          [&]() { return run_degrid(c, image, vis, as_stream(stream)); });
}

wsp_status wsp_grid_ws(wsp_ctx *c, const void *vis, void *image, void *grids, size_t grid_bytes, void *scratch,
                       size_t scratch_bytes, void *stream) {
    if (!c || !image || !vis) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    return with_workspace(c, grids, grid_bytes, scratch, scratch_bytes, "grid",
                          [&]() { return run_grid(c, vis, image, as_stream(stream)); });
}

wsp_status wsp_degrid_pol(wsp_ctx *c, const void *q_image, const void *u_image, void *vis,
                          void *stream) {
    if (!c || !q_image || !u_image || !vis) return fail(WSP_EINVAL, "null argument");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = as_stream(stream);
    HIP_OR_FAIL(run_degrid(c, q_image, vis, s, 0), "degrid (Stokes Q)");
    HIP_OR_FAIL(run_degrid(c, u_image, vis, s, 1), "degrid (Stokes U)");
    return WSP_OK;
}

wsp_status wsp_grid_pol(wsp_ctx *c, const void *vis, void *q_image, void *u_image, void *stream) {
    if (!c || !q_image || !u_image || !vis) return fail(WSP_EINVAL, "null argument");
    if (q_image == u_image) return fail(WSP_EINVAL, "q_image and u_image must differ");
    if (!c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = as_stream(stream);
    HIP_OR_FAIL(run_grid(c, vis, q_image, s, 0), "grid (Stokes Q)");
    HIP_OR_FAIL(run_grid(c, vis, u_image, s, 1), "grid (Stokes U)");
    return WSP_OK;
}

wsp_status wsp_kernel_values(wsp_ctx *c, int64_t p, void *out, int32_t *jp, int32_t *u0,
                             int32_t *v0) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    if (!c->planned) return fail(WSP_ESTATE, "no plan");
    if (out && !c->built) return fail(WSP_ESTATE, "wsp_build_kernels first");
    if (p < 0 || p >= c->plan.m) return fail(WSP_EINVAL, "visibility index out of range");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    TrackScope track(&c->track);
    HIP_OR_FAIL(hipDeviceSynchronize(), "sync");
    int64_t sidx = -1;
    HIP_OR_FAIL(find_sorted_index(c, p, &sidx), "permutation lookup");
    if (sidx < 0) return fail(WSP_EHIP, "permutation lookup failed");
    int32_t j = 0;
    double uu = 0, vv = 0;
    HIP_OR_FAIL(hipMemcpy(&j, c->plan.jp + sidx, sizeof(int32_t), hipMemcpyDeviceToHost), "jp");
    HIP_OR_FAIL(hipMemcpy(&uu, c->plan.u + p, sizeof(double), hipMemcpyDeviceToHost), "u");
    HIP_OR_FAIL(hipMemcpy(&vv, c->plan.v + p, sizeof(double), hipMemcpyDeviceToHost), "v");
    if (jp) *jp = j;
    if (u0) *u0 = (int32_t)((int64_t)std::floor(uu * c->g.inv_du) - j / 2 + 1);
    if (v0) *v0 = (int32_t)((int64_t)std::floor(vv * c->g.inv_du) - j / 2 + 1);
    if (out) {
        const size_t bytes = (size_t)j * j * (c->g.planes ? sizeof(float) * 2 : cplx_bytes(c));
        void *d = nullptr;
        HIP_OR_FAIL(dmalloc(&d, bytes), "hipMalloc");
        hipError_t e = c->g.planes ? run_plane_taps(c, sidx, d, nullptr) : run_exact_taps(c, sidx, d, nullptr);
        if (e == hipSuccess) e = hipMemcpy(out, d, bytes, hipMemcpyDeviceToHost);
        dfree(d);
        if (e != hipSuccess) return hip_fail(e, "kernel taps");
    }
    return WSP_OK;
}

wsp_status wsp_set_timing(wsp_ctx *c, int32_t enable) {
    if (!c) return fail(WSP_EINVAL, "null argument");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    drain_timer(c);
    for (int st = 0; st < kNumStages; ++st) {
        c->timer.ms[st] = 0.0;
        c->timer.count[st] = 0;
    }
    c->timer.enabled = enable != 0;
    return WSP_OK;
}

wsp_status wsp_stage_times(wsp_ctx *c, double *ms, int64_t *counts) {
    if (!c || !ms) return fail(WSP_EINVAL, "null argument");
    HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
    drain_timer(c);
    for (int st = 0; st < kNumStages; ++st) {
        ms[st] = c->timer.ms[st];
        if (counts) counts[st] = c->timer.count[st];
    }
    return WSP_OK;
}

void wsp_destroy(wsp_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    TrackScope track(&c->track);
    drain_timer(c);
    for (hipEvent_t ev : c->timer.pool) hipEventDestroy(ev);
    free_sorted_plan(c->plan);
    free_caller(c->plan);
    dfree(c->dde_u);
    dfree(c->dde_v);
    dfree(c->plan_centres);
    dfree(c->fft_tw);
    if (c->fft_v_made) hipfftDestroy(c->fft_v);
    if (c->fft_u_made) hipfftDestroy(c->fft_u);
    destroy_row_plans(c);
    delete c;
}

}  // extern "C"
