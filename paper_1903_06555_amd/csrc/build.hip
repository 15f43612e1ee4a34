// Kernel builder: one exact w-projection kernel per visibility (Eqs. (5), (6)).
//
//   K_p[row, col] = 2 pi int_0^{alpha/2} g(r) e^{-2 pi i w_eff (n(r) - 1)} J0(2 pi r q) r dr
//
// Visibilities are processed costliest first, in batches: phase 1 runs one
// wavefront per visibility, phase 2 one wavefront per chunk of 512 taps.
//
// Phase 1 (adaptive partition, FP64).  The integrand differs between taps
// only through J0(2 pi r q), so all J_p^2 taps share one panel partition.
// The initial partition holds about one cycle of the integrand's phase bound
// |w| (1 - n(r)) + q_max r per panel.  Each panel is integrated by the
// Gauss-Kronrod (7, 15) pair at kProbes distances q_j spanning [0, q_max];
// its error estimate is max_j |K15_j - G7_j|.  A panel of width h is accepted
// when the estimate is <= tol S h / R, with S the largest |K(q_j)| after the
// first pass (so the panel estimates add up to at most tol S), otherwise it
// is bisected; rounds repeat until every panel passes or the panel cap is
// reached.  Probes are evaluated in FP64 so the estimate is not swamped by
// FP32 rounding, one Gauss-Kronrod node per lane (16-lane groups, four
// panels per pass), the probe sums reduced across each group.
//
// Phase 2 (taps).  Every tap is integrated with the 15-point Kronrod rule on
// the final partition.  FP32 path: node values g(r) r e^{...} in FP64, cast to
// FP32; J0 in FP32 with its phase reduced in FP64; per-panel-group partial
// sums in FP32, accumulated over the partition in FP64.  FP64 path: all FP64.
#include <hipcub/hipcub.hpp>

#include <mutex>
#include <type_traits>

#include "wsp_devmath.h"

namespace wsp {

namespace {

constexpr int kWavesPerBlock = 4;
// taps per lane of the tap kernel: fewer on the FP64 path, whose per-tap
// state is twice as wide, so that more than one wavefront fits per SIMD;
// and fewer when the visibilities have few points each (small supports:
// most lanes' other slots would be idle, and fewer registers per lane let
// more wavefronts hide the latency).  The per-point arithmetic is the same
// either way.
template <bool kFP64, bool kSmall>
constexpr int taps_per_lane() {
    return kSmall ? (kFP64 ? 1 : 2) : (kFP64 ? 4 : 8);
}
// mean points per visibility up to which the small variant runs
constexpr int64_t kSmallTapsPerVis = 256;
constexpr int kPanelGroup = 4;                 // panels per node batch (60 of 64 lanes)
constexpr int kGroupNodes = kPanelGroup * WSP_GK_N;
constexpr int64_t kBuildBatch = 65536;    // visibilities per partition batch

// Radial samples.  K_p depends on a tap only through its distance q, and is
// band-limited (J0(2 pi r q) with r <= alpha / 2): where fewer uniform samples
// q = s h cover a visibility's taps than it has taps, the quadrature runs on
// the samples and each tap is interpolated from the 10 samples around it
// (Lagrange, FP64; K(-q) = K(q) mirrors the first ones).  Measured against
// the oracle at |w| up to 480, the interpolation error is ~3e-9 of the kernel
// peak with h = 1/8 cell (the FP64 path) and ~6e-8 with h = 1/6 (the FP32
// path, whose own rounding is ~1e-7): both far below the 1e-6 quadrature
// tolerance.
constexpr double kSampleStep64 = 0.125, kInvSampleStep64 = 8.0;
constexpr double kSampleStep32 = 1.0 / 6.0, kInvSampleStep32 = 6.0;
constexpr int kStencil = 10;

struct PointSet {
    double qmax;     // largest distance the quadrature must serve
    int64_t npts;    // quadrature points: samples or taps
    bool sampled;
};

// q_max over the J_p x J_p taps at offsets (ux - col, vx - row); samples at
// q = s step
__device__ __forceinline__ PointSet point_set(double ux, double vx, int jp, double step, double inv_step) {
    const double cu = fmax(fabs(ux), fabs(ux - (double)(jp - 1)));
    const double cv = fmax(fabs(vx), fabs(vx - (double)(jp - 1)));
    const double qmax = sqrt(cu * cu + cv * cv);
    // samples 0 .. ns - 1 hold every tap's stencil floor(q / h) - 4 .. floor(q / h) + 5
    const int64_t ns = (int64_t)floor(qmax * inv_step) + kStencil / 2 + 1;
    const int64_t nt = (int64_t)jp * jp;
    if (ns < nt) return {(double)(ns - 1) * step, ns, true};
    return {qmax, nt, false};
}

struct BuildArgs {
    // w-plane mode (plane_off != null): "visibility" j is the plane |w| = j dw,
    // its points the samples q = i dq, written into the pair rows j and j - 1
    const int64_t *plane_off;
    int n_pairs;
    double plane_dq, plane_dw;
    float2 *table2;
    double sstep, inv_sstep;  // radial sample step of the precision path
    // DDE convolution (g.dde_h > 0): per-visibility kernels, caller order, and
    // the sorted -> caller permutation
    const void *dde_u, *dde_v;
    const int32_t *perm;
    const int32_t *border;
    int64_t m;
    const double *ux, *vx, *weff;
    const int32_t *jp;
    const int32_t *u0w, *v0w;
    const int64_t *tap_off;
    TapLayout lay;  // positions of the taps in the band-major layout
    void *taps;
    Geom g;
    double tol;
    int max_panels;
    unsigned long long *stats;
};

// Outer ring of width h of a J_p' x J_p' block: the DDE convolution's margin,
// where the w-kernel itself is zero (Eq. (11)).
__device__ __forceinline__ bool in_dde_ring(int row, int col, int jp, int h) {
    return h > 0 && (row < h || row >= jp - h || col < h || col >= jp - h);
}

// Samples of plane j: as many as the pair row that reads the most of them
// (row j, or row j - 1 for the last plane; rows grow with j).
__device__ __forceinline__ PointSet plane_points(const BuildArgs &A, int j) {
    const int r = j < A.n_pairs ? j : A.n_pairs - 1;
    const int64_t n = A.plane_off[r + 1] - A.plane_off[r];
    return {(double)(n - 1) * A.plane_dq, n, true};
}

// Visibility (or plane) of build slot b, its w_eff and quadrature points.
struct Target {
    int p;
    double weff;
    PointSet ps;
};
__device__ __forceinline__ Target build_target(const BuildArgs &A, int64_t b) {
    if (A.plane_off) {
        const int j = (int)b;
        return {j, (double)j * A.plane_dw, plane_points(A, j)};
    }
    const int p = A.border[b];
    return {p, A.weff[p], point_set(A.ux[p], A.vx[p], A.jp[p], A.sstep, A.inv_sstep)};
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast lane n's value to the wavefront (n wave-uniform).
__device__ __forceinline__ float readlane_f32(float x, int n) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), n));
}
__device__ __forceinline__ double readlane_f64(double x, int n) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), n);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), n);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Integrand phase bound (cycles): |w| (1 - n(r)) + q_max r, increasing in r.
__device__ __forceinline__ double phase_bound(double r, double aw, double qmax, const Geom &g) {
    double rho = r * g.inv_du;
    return aw * (-n_minus_one(rho * rho)) + qmax * r;
}

// Node value 2 pi r g(r) e^{-2 pi i w (n - 1)} in FP64.
__device__ __forceinline__ void node_value(double r, double weff, const Geom &g, double *re,
                                           double *im) {
    double rho = r * g.inv_du;
    double f = reduce_rev(-weff * n_minus_one(rho * rho));
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    double amp = kTwoPi * r * taper_g(r, g);
    *re = amp * cs;
    *im = amp * sn;
}

// Sum over each row of 16 lanes with DPP moves (no LDS): quad swaps, then the
// half-row and row mirrors; every lane of the row ends with the row's sum.
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), kCtrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}

// 1 / j and 1 / sqrt(j) for the probe distances q_j = j q_1: x_j = j x_1, so
// the Hankel factors 8 / x and sqrt(2 / (pi x)) of every probe follow from
// those of probe 1 (one division and one square root per node).
__constant__ double kInvJ[kProbes] = {0.0, 1.0, 0.5, 1.0 / 3.0, 0.25, 0.2, 1.0 / 6.0, 1.0 / 7.0};
__constant__ double kInvSqrtJ[kProbes] = {0.0, 1.0, 0.70710678118654752440, 0.57735026918962576451, 0.5,
                                          0.44721359549995793928, 0.40824829046386301637,
                                          0.37796447300922722721};

// G7/K15 error estimates for the marked panels idx[0 .. ne), one
// Gauss-Kronrod node per lane: 16-lane groups (15 nodes used) take 4 panels
// per pass and sum their nodes across the group, so the per-probe sums live
// across lanes rather than in one lane's registers.  The estimate needs
// only K15 - G7, one sum per probe: max_j |K15_j - G7_j| over the probes.
// Panel idx[k]'s error goes to errv[idx[k]].  With acc (the first round) the
// K15 values are also added into acc[(group * kProbes + j) * 2 + {0, 1}]
// (LDS; each group's first lane owns its entries).
__device__ void eval_marked_grouped(const float *cur, const int *idx, int ne, double weff, double qstep,
                                    const Geom &g, float *errv, double *acc, int lane) {
    const int grp = lane >> 4, nd = lane & 15;
    for (int k0 = 0; k0 < ne; k0 += kWave / 16) {
        const int k = k0 + grp;
        int pi = 0;
        double a = 0.0, b = 0.0;
        if (k < ne) {
            pi = idx[k];
            a = (double)fabsf(cur[pi]);
            b = (double)fabsf(cur[pi + 1]);
        }
        const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
        // idle lanes keep r = 0 and zero weights: they add nothing
        double r = 0.0, are = 0.0, aim = 0.0, wk = 0.0, wg = 0.0, inv1 = 0.0, amp1 = 0.0;
        if (k < ne && nd < WSP_GK_N) {
            r = fma(half, wsp_gk_x[nd], mid);
            node_value(r, weff, g, &are, &aim);
            wk = wsp_gk_wk[nd];
            wg = wsp_gk_wg[nd];
            const double x1 = kTwoPi * (r * qstep);
            inv1 = 8.0 / x1;
            amp1 = sqrt(0.6366197723675814 / x1);
        }
        const double wd = wk - wg;
        double e2 = 0.0;
        // one probe at a time (a rolled loop): fewer live registers
#pragma unroll 1
        for (int j = 0; j < kProbes; ++j) {
            const double q = qstep * j;
            const double x = kTwoPi * (r * q);
            const double J = x < 8.0 ? j0_small(x) : j0_fp64(r, q, inv1 * kInvJ[j], amp1 * kInvSqrtJ[j]);
            const double tr = are * J, ti = aim * J;
            const double dr = row_sum16(wd * tr), di = row_sum16(wd * ti);
            e2 = fmax(e2, dr * dr + di * di);
            if (acc != nullptr) {
                const double kr = row_sum16(wk * tr), ki = row_sum16(wk * ti);
                if (k < ne && nd == 0) {
                    acc[(grp * kProbes + j) * 2] += half * kr;
                    acc[(grp * kProbes + j) * 2 + 1] += half * ki;
                }
            }
        }
        if (k < ne && nd == 0) errv[pi] = (float)(half * sqrt(e2));
    }
}

// Phase 1.  Returns the panel count; the partition ends up in *out (LDS), as
// |bnd[0]| < |bnd[1]| < ... < |bnd[P]|.
__device__ int adaptive_partition(float *bA, float *bB, int *idx, double *acc, float **out, double weff,
                                  double qmax, const BuildArgs &A, int lane, bool *capped) {
    const Geom &g = A.g;
    const double R = g.r_max;
    const double aw = fabs(weff);
    const int cap = A.max_panels;
    double phiR = phase_bound(R, aw, qmax, g);
    int P = (int)ceil(phiR);
    P = P < 2 ? 2 : (P > cap / 2 ? cap / 2 : P);
    // initial boundaries at equal steps of the phase bound (bisection in FP64);
    // negative sign = panel starting here still has to be evaluated
    for (int i = lane; i <= P; i += kWave) {
        float val;
        if (i == 0) {
            val = 0.0f;
        } else if (i == P) {
            val = (float)R;
        } else {
            double target = phiR * (double)i / (double)P;
            double lo = 0.0, hi = R;
            for (int it = 0; it < 48; ++it) {
                double midr = 0.5 * (lo + hi);
                if (phase_bound(midr, aw, qmax, g) < target) lo = midr;
                else hi = midr;
            }
            val = (float)(0.5 * (lo + hi));
        }
        bA[i] = (i < P) ? -val : val;
    }
    wave_sync();
    float *cur = bA, *oth = bB;
    const double qstep = qmax / (double)(kProbes - 1);
    for (int k = lane; k < 2 * 4 * kProbes; k += kWave) acc[k] = 0.0;
    double thr = 0.0;
    *capped = false;
    constexpr int kChunks = kMaxPanels / kWave;
    for (int round = 0; round < 32; ++round) {
        float err[kChunks];
        // panels to evaluate this round (marked by a negative boundary)
        int ne = 0;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (c * kWave < P) {
                const int i = c * kWave + lane;
                ne += __popcll(__ballot(i < P && signbit(cur[i])));
            }
        }
        double *acc_r = round == 0 ? acc : nullptr;
        // errors go through oth: few marked panels are listed and evaluated
        // together, many chunk by chunk
        if (ne <= kWave) {
            int run = 0;
#pragma unroll
            for (int c = 0; c < kChunks; ++c) {
                if (c * kWave < P) {
                    const int i = c * kWave + lane;
                    const bool mk = i < P && signbit(cur[i]);
                    const unsigned long long bal = __ballot(mk);
                    if (mk) idx[run + __popcll(bal & lanemask_lt(lane))] = i;
                    run += __popcll(bal);
                }
            }
            wave_sync();
            eval_marked_grouped(cur, idx, ne, weff, qstep, g, oth, acc_r, lane);
            wave_sync();
        } else {
#pragma unroll 1
            for (int c = 0; c * kWave < P; ++c) {
                const int i = c * kWave + lane;
                const bool mk = i < P && signbit(cur[i]);
                const unsigned long long bal = __ballot(mk);
                if (bal == 0ull) continue;
                if (mk) idx[__popcll(bal & lanemask_lt(lane))] = i;
                wave_sync();
                eval_marked_grouped(cur, idx, __popcll(bal), weff, qstep, g, oth, acc_r, lane);
                wave_sync();  // idx is rewritten by the next chunk
            }
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int i = c * kWave + lane;
            err[c] = (c * kWave < P && i < P && signbit(cur[i])) ? oth[i] : -1.0f;
        }
        wave_sync();  // oth is rewritten by the split below
        if (round == 0) {
            // S = max_j |K(q_j)| from the first pass over the whole interval
            double S = 0.0;
#pragma unroll
            for (int j = 0; j < kProbes; ++j) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int gq = 0; gq < 4; ++gq) {
                    re += acc[(gq * kProbes + j) * 2];
                    im += acc[(gq * kProbes + j) * 2 + 1];
                }
                S = fmax(S, sqrt(re * re + im * im));
            }
            thr = A.tol * S / R;
        }
        // count the panels to split; a panel over the tolerance but too narrow
        // to split (FP32 boundaries) stays whole and marks the visibility capped
        int total = 0;
        bool floor_hit = false;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (c * kWave < P) {
                int i = c * kWave + lane;
                bool sp = false, over = false;
                if (i < P && err[c] >= 0.0f) {
                    float wa = fabsf(cur[i]), wb = fabsf(cur[i + 1]);
                    over = (double)err[c] > thr * (double)(wb - wa);
                    sp = over && (wb - wa) > 4.0e-6f * wb;
                }
                total += __popcll(__ballot(sp));
                floor_hit = floor_hit || __ballot(over && !sp) != 0ull;
            }
        }
        if (floor_hit) *capped = true;
        if (total == 0) break;
        if (P + total > cap) {
            *capped = true;
            break;
        }
        // rebuild the boundary list with the midpoints inserted
        int run = 0;
#pragma unroll
        for (int c = 0; c <= kChunks; ++c) {
            if (c * kWave <= P) {
                int i = c * kWave + lane;
                bool sp = false;
                float wa = 0.0f, wb = 0.0f;
                if (i < P && c < kChunks && err[c] >= 0.0f) {
                    wa = fabsf(cur[i]);
                    wb = fabsf(cur[i + 1]);
                    sp = (double)err[c] > thr * (double)(wb - wa) && (wb - wa) > 4.0e-6f * wb;
                }
                unsigned long long bal = __ballot(sp);
                int pre = run + __popcll(bal & lanemask_lt(lane));
                if (i <= P) {
                    float v = fabsf(cur[i]);
                    oth[i + pre] = (sp && i < P) ? -v : v;
                    if (sp) oth[i + pre + 1] = -(0.5f * (wa + wb));
                }
                run += __popcll(bal);
            }
        }
        wave_sync();
        float *t = cur;
        cur = oth;
        oth = t;
        P += total;
    }
    *out = cur;
    return P;
}

// Phase 1 kernel: one wavefront per visibility of the batch; writes the
// final partition (|boundaries|) and its panel count.  Register use is
// capped for three wavefronts per SIMD (168 VGPRs, a few bytes of spill).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_partition(
    BuildArgs A, int64_t batch0, int nb, float *part, int *npan) {
    __shared__ float s_bnd[kWavesPerBlock][2][kMaxPanels + 2];
    __shared__ int s_idx[kWavesPerBlock][kWave];
    __shared__ double s_acc[kWavesPerBlock][2 * 4 * kProbes];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int i = blockIdx.x * kWavesPerBlock + wid;
    if (i >= nb) return;  // whole wave leaves; no block-wide barriers below
    const Target tg = build_target(A, batch0 + i);
    const double weff = tg.weff, qmax = tg.ps.qmax;
    float *bnd = nullptr;
    bool capped = false;
    int P = adaptive_partition(s_bnd[wid][0], s_bnd[wid][1], s_idx[wid], s_acc[wid], &bnd, weff, qmax, A, lane,
                               &capped);
    float *dst = part + (int64_t)i * (kMaxPanels + 2);
    for (int k = lane; k <= P; k += kWave) dst[k] = fabsf(bnd[k]);
    if (lane == 0) {
        npan[i] = P;
        atomicAdd(&A.stats[0], (unsigned long long)P);
        if (capped) atomicAdd(&A.stats[1], 1ull);
    }
}

// Phase 2 kernel: one wavefront per (visibility, chunk of 64 x
// taps_per_lane quadrature points); unit_off is the exclusive prefix of
// chunks per visibility.  The points are the visibility's taps, or its
// radial samples (then written, in FP64, to samples + samp_off[i]).
template <bool kFP64, bool kSmall>
__global__ __launch_bounds__(256) void k_taps(BuildArgs A, int64_t batch0, int nb,
                                              const float *__restrict__ part,
                                              const int *__restrict__ npan,
                                              const int *__restrict__ unit_off, int nunits,
                                              double2 *samples, const int64_t *__restrict__ samp_off) {
    constexpr int kTapsPerLane = taps_per_lane<kFP64, kSmall>();
    const int lane = threadIdx.x & (kWave - 1);
    const int unit = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (unit >= nunits) return;
    // visibility of this unit: last i with unit_off[i] <= unit
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (unit_off[mid] <= unit) lo = mid;
        else hi = mid - 1;
    }
    const int i = lo;
    const Geom &g = A.g;
    const Target tg = build_target(A, batch0 + i);
    const int p = tg.p;
    const bool planes = A.plane_off != nullptr;
    const double ux = planes ? 0.0 : A.ux[p], vx = planes ? 0.0 : A.vx[p], weff = tg.weff;
    const int jp = planes ? 1 : A.jp[p];
    const PointSet ps = tg.ps;
    const int64_t ntap = ps.npts;
    const double sstep = planes ? A.plane_dq : A.sstep;
    const int P = npan[i];
    const float *bnd = part + (int64_t)i * (kMaxPanels + 2);
    const int64_t chunk = (int64_t)kWave * kTapsPerLane;
    const int64_t cbase = (int64_t)(unit - unit_off[i]) * chunk;

    double q[kTapsPerLane];
    float qf[kTapsPerLane], qinv[kTapsPerLane];
    double qinv64[kTapsPerLane], qrs64[kTapsPerLane];
    double accr[kTapsPerLane], acci[kTapsPerLane];
#pragma unroll
    for (int k = 0; k < kTapsPerLane; ++k) {
        int64_t t = cbase + (int64_t)k * kWave + lane;
        int row = (int)(t / jp);
        int col = (int)(t - (int64_t)row * jp);
        double du = ux - (double)col, dv = vx - (double)row;
        q[k] = (t < ntap) ? (ps.sampled ? (double)t * sstep : sqrt(du * du + dv * dv)) : 0.0;
        qf[k] = (float)(kTwoPi * q[k]);
        // per-tap factors of 8 / x and sqrt(2 / (pi x)) (unused when q = 0)
        qinv[k] = q[k] > 0.0 ? (float)(1.0 / q[k]) : 0.0f;
        qrs64[k] = q[k] > 0.0 ? 1.0 / sqrt(q[k]) : 0.0;
        if constexpr (kFP64) qinv64[k] = q[k] > 0.0 ? 1.0 / q[k] : 0.0;
        accr[k] = acci[k] = 0.0;
    }
    for (int pg = 0; pg < P; pg += kPanelGroup) {
        // node data for kPanelGroup panels: lane = panel * 15 + node
        double nr = 0.0, nre = 0.0, nim = 0.0;
        {
            int pan = pg + lane / WSP_GK_N;
            int nd = lane % WSP_GK_N;
            if (lane < kGroupNodes && pan < P) {
                double a = (double)bnd[pan], b = (double)bnd[pan + 1];
                double half = 0.5 * (b - a);
                nr = fma(half, wsp_gk_x[nd], 0.5 * (a + b));
                node_value(nr, weff, g, &nre, &nim);
                double wgt = half * wsp_gk_wk[nd];
                nre *= wgt;
                nim *= wgt;
            }
        }
        const int nn = (P - pg >= kPanelGroup ? kPanelGroup : P - pg) * WSP_GK_N;
        if constexpr (kFP64) {
            // per-node factors of 8 / x and sqrt(2 / (pi x)), as in the FP32 branch
            const double rinv64 = nr > 0.0 ? 1.2732395447351627 / nr : 0.0;
            const double rrs64 = nr > 0.0 ? 0.3183098861837907 / sqrt(nr) : 0.0;
            double pr[kTapsPerLane], pi_[kTapsPerLane];
#pragma unroll
            for (int k = 0; k < kTapsPerLane; ++k) pr[k] = pi_[k] = 0.0;
            for (int n = 0; n < nn; ++n) {
                const double rn = readlane_f64(nr, n);
                const double are = readlane_f64(nre, n), aim = readlane_f64(nim, n);
                const double ri = readlane_f64(rinv64, n), rr = readlane_f64(rrs64, n);
#pragma unroll
                for (int k = 0; k < kTapsPerLane; ++k) {
                    if (cbase + (int64_t)k * kWave < ntap) {
                        double J = j0_fp64(rn, q[k], ri * qinv64[k], rr * qrs64[k]);
                        pr[k] = fma(are, J, pr[k]);
                        pi_[k] = fma(aim, J, pi_[k]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kTapsPerLane; ++k) {
                accr[k] += pr[k];
                acci[k] += pi_[k];
            }
        } else {
            // per-node factors, broadcast with readlane (no LDS round trip); the
            // node weights, the Bessel amplitude and the sums stay in FP64
            const float rinv = nr > 0.0 ? (float)(1.2732395447351627 / nr) : 0.0f;  // (4/pi) / r
            const double rrs = nr > 0.0 ? 0.3183098861837907 / sqrt(nr) : 0.0;     // 1 / (pi sqrt r)
            const float nrf = (float)nr;
            for (int n = 0; n < nn; ++n) {
                const double rn = readlane_f64(nr, n);
                const double are = readlane_f64(nre, n), aim = readlane_f64(nim, n);
                const float ri = readlane_f32(rinv, n);
                const double rr = readlane_f64(rrs, n);
                const float rnf = readlane_f32(nrf, n);
#pragma unroll
                for (int k = 0; k < kTapsPerLane; ++k) {
                    if (cbase + (int64_t)k * kWave < ntap) {
                        const double J = j0_fp64phase(rn, q[k], rnf * qf[k], ri * qinv[k], rr * qrs64[k]);
                        accr[k] = fma(are, J, accr[k]);
                        acci[k] = fma(aim, J, acci[k]);
                    }
                }
            }
        }
    }
    if (planes) {
        // sample t of plane j: T[j, t] of pair row j and T[j, t] of row j - 1
        const int64_t n_lo = p < A.n_pairs ? A.plane_off[p + 1] - A.plane_off[p] : 0;
        const int64_t n_hi = p >= 1 ? A.plane_off[p] - A.plane_off[p - 1] : 0;
#pragma unroll
        for (int k = 0; k < kTapsPerLane; ++k) {
            const int64_t t = cbase + (int64_t)k * kWave + lane;
            const float2 v = make_float2((float)accr[k], (float)acci[k]);
            if (t < n_lo) A.table2[2 * (A.plane_off[p] + t)] = v;
            if (t < n_hi) A.table2[2 * (A.plane_off[p - 1] + t) + 1] = v;
        }
        return;
    }
    if (ps.sampled) {
        double2 *dst = samples + samp_off[i];
#pragma unroll
        for (int k = 0; k < kTapsPerLane; ++k) {
            const int64_t t = cbase + (int64_t)k * kWave + lane;
            if (t < ntap) dst[t] = make_double2(accr[k], acci[k]);
        }
        return;
    }
    const int u0w = A.u0w[p], v0w = A.v0w[p];
#pragma unroll
    for (int k = 0; k < kTapsPerLane; ++k) {
        int64_t t = cbase + (int64_t)k * kWave + lane;
        if (t < ntap) {
            const int row = (int)(t / jp), col = (int)(t - (int64_t)(t / jp) * jp);
            const int64_t pos = tap_position(A.lay, p, row, col, jp, u0w, v0w);
            // with a DDE convolution the w-kernel fills the inner block only
            const bool ring = in_dde_ring(row, col, jp, g.dde_h);
            if constexpr (kFP64) {
                ((double2 *)A.taps)[pos] = ring ? make_double2(0.0, 0.0) : make_double2(accr[k], acci[k]);
            } else {
                ((float2 *)A.taps)[pos] = ring ? make_float2(0.0f, 0.0f)
                                               : make_float2((float)accr[k], (float)acci[k]);
            }
        }
    }
}

// Tap values of the sampled visibilities of a batch: one block per visibility,
// each tap interpolated from the 10 radial samples around its distance.
template <bool kFP64>
__global__ __launch_bounds__(256) void k_interp(BuildArgs A, int64_t batch0,
                                                const double2 *__restrict__ samples,
                                                const int64_t *__restrict__ samp_off) {
    const int i = blockIdx.x;
    const int p = A.border[batch0 + i];
    const double ux = A.ux[p], vx = A.vx[p];
    const int jp = A.jp[p];
    const PointSet ps = point_set(ux, vx, jp, A.sstep, A.inv_sstep);
    if (!ps.sampled) return;  // uniform over the block
    const double2 *smp = samples + samp_off[i];
    const int u0w = A.u0w[p], v0w = A.v0w[p];
    const int64_t ntap = (int64_t)jp * jp;
    for (int64_t t = threadIdx.x; t < ntap; t += blockDim.x) {
        const int row = (int)(t / jp), col = (int)(t - (int64_t)row * jp);
        const double du = ux - (double)col, dv = vx - (double)row;
        const double x = sqrt(du * du + dv * dv) * A.inv_sstep;
        const int s0 = (int)floor(x) - (kStencil / 2 - 1);
        const double u = x - (double)s0;  // in [4, 5): position inside the stencil
        // Lagrange basis on the nodes 0 .. 9: l_k(u) = c_k prod_{j != k} (u - j),
        // c_k = (-1)^(9 - k) / (k! (9 - k)!)
        double pre[kStencil], suf[kStencil];
        pre[0] = 1.0;
#pragma unroll
        for (int k = 1; k < kStencil; ++k) pre[k] = pre[k - 1] * (u - (double)(k - 1));
        suf[kStencil - 1] = 1.0;
#pragma unroll
        for (int k = kStencil - 2; k >= 0; --k) suf[k] = suf[k + 1] * (u - (double)(k + 1));
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int k = 0; k < kStencil; ++k) {
            const int sidx = s0 + k;
            const double2 v = smp[sidx < 0 ? -sidx : sidx];
            const double lk = wsp_lagrange10_c[k] * pre[k] * suf[k];
            re = fma(lk, v.x, re);
            im = fma(lk, v.y, im);
        }
        const int64_t pos = tap_position(A.lay, p, row, col, jp, u0w, v0w);
        if (in_dde_ring(row, col, jp, A.g.dde_h)) re = im = 0.0;
        if constexpr (kFP64) {
            ((double2 *)A.taps)[pos] = make_double2(re, im);
        } else {
            ((float2 *)A.taps)[pos] = make_float2((float)re, (float)im);
        }
    }
}

// DDE convolution of the built taps of a batch (Eq. (11)), one wavefront per
// visibility, in place: K'[r, c] = sum_b d_v[b] H[r - b, c] with
// H[r, c] = sum_a d_u[a] K[r, c - a] (a, b in -h .. h, out-of-block terms 0).
// Row r of K is overwritten at step r; H row r + h is formed at step r from
// K row r + h (not yet overwritten) into a ring of 2h + 1 rows in LDS, which
// then holds every H row that output row r needs.
template <bool kFP64>
__global__ __launch_bounds__(64) void k_dde_conv(BuildArgs A, int64_t batch0) {
    using C = typename std::conditional<kFP64, double2, float2>::type;
    extern __shared__ char dde_lds[];
    C *ring = (C *)dde_lds;
    const int h = A.g.dde_h, JD = 2 * h + 1;
    const int p = A.border[batch0 + blockIdx.x];
    const int J = A.jp[p];
    const int64_t cp = A.perm[p];
    const C *du = (const C *)A.dde_u + cp * JD;
    const C *dv = (const C *)A.dde_v + cp * JD;
    C *taps = (C *)A.taps;
    const int u0w = A.u0w[p], v0w = A.v0w[p];
    const int lane = threadIdx.x;
    for (int r = -h; r < J; ++r) {
        const int hr = r + h;  // H row formed at this step
        C *slot = ring + (int64_t)(hr % JD) * J;
        for (int c = lane; c < J; c += 64) {
            C acc;
            acc.x = 0;
            acc.y = 0;
            if (hr < J) {
                for (int a = -h; a <= h; ++a) {
                    const int cc = c - a;
                    if (cc < 0 || cc >= J) continue;
                    const C k = taps[tap_position(A.lay, p, hr, cc, J, u0w, v0w)];
                    const C d = du[a + h];
                    acc.x += d.x * k.x - d.y * k.y;
                    acc.y += d.x * k.y + d.y * k.x;
                }
            }
            slot[c] = acc;
        }
        __syncthreads();
        if (r >= 0) {
            for (int c = lane; c < J; c += 64) {
                C acc;
                acc.x = 0;
                acc.y = 0;
                for (int b = -h; b <= h; ++b) {
                    const int rr = r - b;
                    if (rr < 0 || rr >= J) continue;
                    const C hv = ring[(int64_t)(rr % JD) * J + c];
                    const C d = dv[b + h];
                    acc.x += d.x * hv.x - d.y * hv.y;
                    acc.y += d.x * hv.y + d.y * hv.x;
                }
                taps[tap_position(A.lay, p, r, c, J, u0w, v0w)] = acc;
            }
        }
        __syncthreads();
    }
}

// Per visibility of the batch: quadrature chunks (cnt) and radial samples (scnt).
__global__ void k_unit_counts(BuildArgs A, int64_t batch0, int nb, int64_t chunk, int *cnt,
                              int64_t *scnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nb) return;
    if (i == nb) {
        cnt[i] = 0;
        scnt[i] = 0;
        return;
    }
    const PointSet ps = build_target(A, batch0 + i).ps;
    cnt[i] = (int)((ps.npts + chunk - 1) / chunk);
    scnt[i] = (ps.sampled && !A.plane_off) ? ps.npts : 0;  // plane samples go to the lattice
}

}  // namespace

namespace {

// ---- build workspace -------------------------------------------------------
// The temporaries of one build batch of B visibilities: the partitions
// (kMaxPanels + 2 boundaries each), panel counts, per-visibility unit and
// sample counts with their exclusive scans (and the scans' hipcub storage),
// and the FP64 radial samples.  They come either from hipMalloc (one
// allocation per array, freed at the end of the build) or from one region
// given by the caller of run_build, carved at 256-byte boundaries.

constexpr size_t kWsAlign = 256;

size_t ws_round(size_t x) { return (x + kWsAlign - 1) & ~(kWsAlign - 1); }

// Upper bound on the radial samples of one visibility of support jp: samples
// are used only below jp^2 points, and their count is floor(q_max / h) + 6
// with q_max <= jp / sqrt(2) (the visibility sits within half a cell of its
// support's centre).
int64_t max_samples_per_vis(int jp, double inv_step) {
    const int64_t ns = (int64_t)floor((double)jp * 0.70710678118654757 * inv_step) + kStencil / 2 + 2;
    const int64_t nt = (int64_t)jp * jp;
    return ns < nt ? ns : nt;
}

struct WsLayout {
    size_t part, npan, cnt, scnt, soff, uoff, tmp, tmp2, samples, total;
};

// Byte layout of the temporaries for batches of B visibilities with at most
// `samples` radial samples per batch.  The hipcub storage sizes come from
// hipcub's own size queries (no allocation).
hipError_t ws_layout(int B, int64_t samples, WsLayout *L) {
    size_t tmp = 0, tmp2 = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, (const int *)nullptr, (int *)nullptr, B + 1);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp2, (const int64_t *)nullptr, (int64_t *)nullptr, B + 1);
    if (e != hipSuccess) return e;
    L->part = ws_round(sizeof(float) * (size_t)B * (kMaxPanels + 2));
    L->npan = ws_round(sizeof(int) * (size_t)B);
    L->cnt = ws_round(sizeof(int) * (size_t)(B + 1));
    L->scnt = ws_round(sizeof(int64_t) * (size_t)(B + 1));
    L->soff = ws_round(sizeof(int64_t) * (size_t)(B + 1));
    L->uoff = ws_round(sizeof(int) * (size_t)(B + 1));
    L->tmp = ws_round(tmp > 0 ? tmp : 1);
    L->tmp2 = ws_round(tmp2 > 0 ? tmp2 : 1);
    L->samples = ws_round(sizeof(double2) * (size_t)(samples > 0 ? samples : 1));
    L->total = L->part + L->npan + L->cnt + L->scnt + L->soff + L->uoff + L->tmp + L->tmp2 + L->samples;
    return hipSuccess;
}

// Largest radial-sample count a batch of B build slots can need (w-plane
// samples are written to the lattice directly).
int64_t batch_samples_bound(const wsp_ctx *c, bool planes, double inv_step, int B) {
    if (planes) return 0;
    return (int64_t)B * max_samples_per_vis(c->plan.max_jp, inv_step);
}

// Batch size of a build that must fit `cap` bytes of workspace (0 if not even
// one visibility fits).
hipError_t fitting_batch(const wsp_ctx *c, const BuildArgs &A, int64_t count, size_t cap, int *B_out) {
    int B = (int)(count < kBuildBatch ? count : kBuildBatch);
    while (B >= 1) {
        WsLayout L;
        hipError_t e = ws_layout(B, batch_samples_bound(c, A.plane_off != nullptr, A.inv_sstep, B), &L);
        if (e != hipSuccess) return e;
        if (L.total <= cap) break;
        // shrink in proportion to the overshoot (at least by one)
        const int nb = (int)((double)B * (double)cap / (double)L.total * 0.98);
        B = nb < B ? nb : B - 1;
    }
    *B_out = B > 0 ? B : 0;
    return hipSuccess;
}

// Phases 1 and 2 over build slots first .. first + count - 1, in batches.
// ws == nullptr: the temporaries are allocated with hipMalloc and freed on
// return.  Otherwise they are carved from [ws, ws + ws_bytes) and nothing is
// allocated; the batch size is then the largest whose worst case fits.
hipError_t run_build(wsp_ctx *c, const BuildArgs &A, int64_t first, int64_t count, hipStream_t s,
                     char *ws = nullptr, size_t ws_bytes = 0) {
    const Plan &pl = c->plan;
    hipError_t e = hipSuccess;
    if (first == 0) {
        e = hipMemsetAsync(pl.stats, 0, 2 * sizeof(unsigned long long), s);
        if (e != hipSuccess) return e;
    }
    const int64_t end = first + count;
    int B = (int)(count < kBuildBatch ? count : kBuildBatch);
    if (ws) {
        e = fitting_batch(c, A, count, ws_bytes, &B);
        if (e != hipSuccess) return e;
        if (B < 1) return hipErrorOutOfMemory;
    }
    float *part = nullptr;
    int *npan = nullptr, *cnt = nullptr, *uoff = nullptr;
    int64_t *scnt = nullptr, *soff = nullptr;
    double2 *samples = nullptr;
    int64_t samples_cap = 0;
    void *tmp2 = nullptr;
    size_t tmp2_bytes = 0;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    auto cleanup = [&]() {
        if (ws) return;  // carved from the caller's region: nothing to free
        dfree(part);
        dfree(npan);
        dfree(cnt);
        dfree(uoff);
        dfree(scnt);
        dfree(soff);
        dfree(samples);
        dfree(tmp2);
        dfree(tmp);
    };
#define WSP_BSTEP(expr)        \
    do {                       \
        e = (expr);            \
        if (e != hipSuccess) { \
            cleanup();         \
            return e;          \
        }                      \
    } while (0)
    if (ws) {
        WsLayout L;
        WSP_BSTEP(ws_layout(B, batch_samples_bound(c, A.plane_off != nullptr, A.inv_sstep, B), &L));
        char *q = ws;
        part = (float *)q;
        q += L.part;
        npan = (int *)q;
        q += L.npan;
        cnt = (int *)q;
        q += L.cnt;
        scnt = (int64_t *)q;
        q += L.scnt;
        soff = (int64_t *)q;
        q += L.soff;
        uoff = (int *)q;
        q += L.uoff;
        tmp = q;
        tmp_bytes = L.tmp;
        q += L.tmp;
        tmp2 = q;
        tmp2_bytes = L.tmp2;
        q += L.tmp2;
        samples = (double2 *)q;
        samples_cap = (int64_t)(L.samples / sizeof(double2));
    } else {
        WSP_BSTEP(dmalloc(&part, sizeof(float) * (size_t)B * (kMaxPanels + 2)));
        WSP_BSTEP(dmalloc(&npan, sizeof(int) * (size_t)B));
        WSP_BSTEP(dmalloc(&cnt, sizeof(int) * (size_t)(B + 1)));
        WSP_BSTEP(dmalloc(&scnt, sizeof(int64_t) * (size_t)(B + 1)));
        WSP_BSTEP(dmalloc(&soff, sizeof(int64_t) * (size_t)(B + 1)));
        WSP_BSTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp2_bytes, scnt, soff, B + 1, s));
        WSP_BSTEP(dmalloc(&tmp2, tmp2_bytes));
        WSP_BSTEP(dmalloc(&uoff, sizeof(int) * (size_t)(B + 1)));
        WSP_BSTEP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, uoff, B + 1, s));
        WSP_BSTEP(dmalloc(&tmp, tmp_bytes));
    }
    const bool small = pl.total_taps <= kSmallTapsPerVis * pl.m;
    for (int64_t b0 = first; b0 < end; b0 += B) {
        int nb = (int)(end - b0 < B ? end - b0 : B);
        dim3 block(kWave * kWavesPerBlock);
        hipLaunchKernelGGL(k_partition, dim3((nb + kWavesPerBlock - 1) / kWavesPerBlock), block, 0,
                           s, A, b0, nb, part, npan);
        const int64_t chunk =
            (int64_t)kWave * (c->p.precision == WSP_FP64 ? (small ? taps_per_lane<true, true>() : taps_per_lane<true, false>())
                                                         : (small ? taps_per_lane<false, true>() : taps_per_lane<false, false>()));
        hipLaunchKernelGGL(k_unit_counts, dim3((nb + 1 + 255) / 256), dim3(256), 0, s, A, b0, nb,
                           chunk, cnt, scnt);
        WSP_BSTEP(hipGetLastError());
        WSP_BSTEP(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, uoff, nb + 1, s));
        WSP_BSTEP(hipcub::DeviceScan::ExclusiveSum(tmp2, tmp2_bytes, scnt, soff, nb + 1, s));
        int nunits = 0;
        int64_t nsamp = 0;
        WSP_BSTEP(hipMemcpyAsync(&nunits, uoff + nb, sizeof(int), hipMemcpyDeviceToHost, s));
        WSP_BSTEP(hipMemcpyAsync(&nsamp, soff + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        WSP_BSTEP(hipStreamSynchronize(s));  // also: the previous batch no longer uses samples
        if (nsamp > samples_cap) {
            if (ws) {  // cannot happen: the layout holds the worst case
                e = hipErrorOutOfMemory;
                cleanup();
                return e;
            }
            dfree(samples);
            samples = nullptr;
            samples_cap = 0;
            WSP_BSTEP(dmalloc(&samples, sizeof(double2) * (size_t)nsamp));
            samples_cap = nsamp;
        }
        dim3 grid((unsigned)((nunits + kWavesPerBlock - 1) / kWavesPerBlock));
        if (c->p.precision == WSP_FP64) {
            if (small)
                hipLaunchKernelGGL((k_taps<true, true>), grid, block, 0, s, A, b0, nb, part, npan, uoff, nunits,
                                   samples, soff);
            else
                hipLaunchKernelGGL((k_taps<true, false>), grid, block, 0, s, A, b0, nb, part, npan, uoff, nunits,
                                   samples, soff);
            if (nsamp > 0)
                hipLaunchKernelGGL(k_interp<true>, dim3(nb), dim3(256), 0, s, A, b0,
                                   (const double2 *)samples, soff);
        } else {
            if (small)
                hipLaunchKernelGGL((k_taps<false, true>), grid, block, 0, s, A, b0, nb, part, npan, uoff,
                                   nunits, samples, soff);
            else
                hipLaunchKernelGGL((k_taps<false, false>), grid, block, 0, s, A, b0, nb, part, npan, uoff,
                                   nunits, samples, soff);
            if (nsamp > 0)
                hipLaunchKernelGGL(k_interp<false>, dim3(nb), dim3(256), 0, s, A, b0,
                                   (const double2 *)samples, soff);
        }
        WSP_BSTEP(hipGetLastError());
        if (A.g.dde_h > 0 && !A.plane_off) {
            const size_t lds = (size_t)(2 * A.g.dde_h + 1) * pl.max_jp * cplx_bytes(c);
            if (c->p.precision == WSP_FP64)
                hipLaunchKernelGGL(k_dde_conv<true>, dim3(nb), dim3(64), lds, s, A, b0);
            else
                hipLaunchKernelGGL(k_dde_conv<false>, dim3(nb), dim3(64), lds, s, A, b0);
            WSP_BSTEP(hipGetLastError());
        }
    }
    WSP_BSTEP(hipStreamSynchronize(s));
    cleanup();
    return hipSuccess;
#undef WSP_BSTEP
}

BuildArgs common_args(wsp_ctx *c) {
    BuildArgs A{};
    A.g = c->g;
    // both tolerances are relative to the visibility's kernel peak: the
    // tighter positive one decides
    const double ta = c->p.quad_abs_tol, tr = c->p.quad_rel_tol;
    A.tol = (ta > 0.0 && tr > 0.0) ? (ta < tr ? ta : tr) : (ta > 0.0 ? ta : tr);
    A.max_panels = c->p.quad_max_panels;
    A.stats = c->plan.stats;
    const bool fp64 = c->p.precision == WSP_FP64;
    A.sstep = fp64 ? kSampleStep64 : kSampleStep32;
    A.inv_sstep = fp64 ? kInvSampleStep64 : kInvSampleStep32;
    return A;
}

}  // namespace

hipError_t launch_build(wsp_ctx *c, int64_t first, int64_t count, hipStream_t s, void *ws, size_t ws_bytes) {
    BuildArgs A = common_args(c);
    const Plan &pl = c->plan;
    A.border = pl.border;
    A.m = pl.m;
    A.ux = pl.ux;
    A.vx = pl.vx;
    A.weff = pl.weff;
    A.jp = pl.jp;
    A.u0w = pl.u0w;
    A.v0w = pl.v0w;
    A.tap_off = pl.tap_off;
    A.lay = tap_layout(pl);
    A.taps = c->taps;
    A.dde_u = c->dde_u;
    A.dde_v = c->dde_v;
    A.perm = pl.perm;
    return run_build(c, A, first, count, s, (char *)ws, ws_bytes);
}

// The w-plane lattice: planes j = 0 .. n_pairs (|w| = j dw), FP32 quadrature path.
hipError_t launch_plane_build(wsp_ctx *c, hipStream_t s, void *ws, size_t ws_bytes) {
    BuildArgs A = common_args(c);
    const Plan &pl = c->plan;
    A.plane_off = pl.plane_off;
    A.n_pairs = pl.n_pairs;
    A.plane_dq = c->g.plane_dq;
    A.plane_dw = c->g.plane_dw;
    A.table2 = (float2 *)c->taps;
    return run_build(c, A, 0, (int64_t)pl.n_pairs + 1, s, (char *)ws, ws_bytes);
}

// Batch size of a build whose temporaries must fit `cap` bytes (0: none fits).
int build_batch_in(const wsp_ctx *c, size_t cap) {
    BuildArgs A = common_args(const_cast<wsp_ctx *>(c));
    if (c->g.planes) A.plane_off = c->plan.plane_off;
    const int64_t count = c->g.planes ? (int64_t)c->plan.n_pairs + 1 : c->plan.m;
    int B = 0;
    if (fitting_batch(c, A, count, cap, &B) != hipSuccess) return 0;
    return B;
}

// Peak bytes the allocating build holds at once (its batch temporaries).
size_t build_temp_bytes(const wsp_ctx *c) {
    const BuildArgs A = common_args(const_cast<wsp_ctx *>(c));
    const int64_t count = c->g.planes ? (int64_t)c->plan.n_pairs + 1 : c->plan.m;
    const int B = (int)(count < kBuildBatch ? count : kBuildBatch);
    WsLayout L;
    if (ws_layout(B, batch_samples_bound(c, c->g.planes, A.inv_sstep, B), &L) != hipSuccess) return 0;
    return L.total;
}

// ---- static build workspace ----------------------------------------------------------
// For callers that cannot allocate device memory (graph capture, tight
// serving loops): wsp_build_kernels_noalloc carves the build temporaries
// from this array instead of hipMalloc.  Every device that loads the library
// holds its own copy until the process ends.  Its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) when a
// context is created there; host code uses only that address.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch_init(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // callers make `device` current first
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace wsp
