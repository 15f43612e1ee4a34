// w-plane mode (Sec. 5.1.1): kernel taps interpolated bilinearly from the
// lattice T[j, i] = K(i dq, j dw) of Eq. (6), q, w >= 0.
//
// The lattice is stored as pair rows: row j holds float4 (T[j, i], T[j+1, i])
// (complex64 each), so one 16-byte load fetches both planes around a
// visibility's |w_eff|, and a tap needs two loads (columns i and i + 1).
// Pair row j starts at plane_off[j] (float4 units) and serves
// j dw <= |w_eff| < (j + 1) dw.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wsp {

// Plane record of a visibility (|w_eff| -> pair row, upper-plane weight s,
// conjugation for w_eff < 0) seen from a tap sub-block whose first tap is
// (dx0, dy0) cells away from the visibility.  Packed as
// {row start, last usable column | conj << 31, dx0 bits, dy0 bits} and s.
__device__ __forceinline__ void plane_record(double weff, double dx0, double dy0,
                                             const int64_t *__restrict__ plane_off, int n_pairs,
                                             double inv_dw, int4 *rec, float *sw) {
    const double a = fabs(weff) * inv_dw;
    int j = (int)floor(a);
    j = j < 0 ? 0 : (j > n_pairs - 1 ? n_pairs - 1 : j);
    const double s = fmin(fmax(a - (double)j, 0.0), 1.0);
    const int64_t o = plane_off[j];
    const int nmax = (int)(plane_off[j + 1] - o) - 2;  // columns i and i + 1 stay inside the row
    *rec = make_int4((int)o, nmax | (weff < 0.0 ? (int)0x80000000u : 0), __float_as_int((float)dx0),
                     __float_as_int((float)dy0));
    *sw = (float)s;
}

struct PlaneEntry {
    const float4 *row;
    int nmax;
    float dx0, dy0;  // visibility minus the sub-block's first tap (cells)
    float sw;        // weight of plane j + 1
    float sgn;       // -1: conjugate (w_eff < 0)
};

__device__ __forceinline__ PlaneEntry plane_entry(int4 r, float sw, const float4 *table) {
    PlaneEntry e;
    e.row = table + r.x;
    e.nmax = r.y & 0x7FFFFFFF;
    e.sgn = r.y < 0 ? -1.0f : 1.0f;
    e.dx0 = __int_as_float(r.z);
    e.dy0 = __int_as_float(r.w);
    e.sw = sw;
    return e;
}

// The two lattice columns around x = q / dq of sub-block tap (row, col), and
// the position t in between.  Loads are issued here and consumed by
// plane_value, so a batch of taps keeps its loads in flight together.
struct PlaneLoad {
    float4 a, b;
    float t;
};

__device__ __forceinline__ PlaneLoad plane_load(const PlaneEntry &e, int row, int col, float inv_dq) {
    const float dx = e.dx0 - (float)col, dy = e.dy0 - (float)row;
    const float x = sqrtf(fmaf(dx, dx, dy * dy)) * inv_dq;
    int i = (int)x;
    i = i < e.nmax ? i : e.nmax;
    PlaneLoad l;
    l.t = fminf(x - (float)i, 1.0f);
    l.a = e.row[i];
    l.b = e.row[i + 1];
    return l;
}

__device__ __forceinline__ PlaneLoad plane_zero() {
    PlaneLoad l;
    l.a = make_float4(0.f, 0.f, 0.f, 0.f);
    l.b = l.a;
    l.t = 0.f;
    return l;
}

// (1 - s)[(1 - t) T[j, i] + t T[j, i+1]] + s[(1 - t) T[j+1, i] + t T[j+1, i+1]], conjugated if sgn < 0
__device__ __forceinline__ float2 plane_value(const PlaneLoad &l, float sw, float sgn) {
    const float lr = fmaf(sw, l.a.z - l.a.x, l.a.x), li = fmaf(sw, l.a.w - l.a.y, l.a.y);
    const float hr = fmaf(sw, l.b.z - l.b.x, l.b.x), hi = fmaf(sw, l.b.w - l.b.y, l.b.y);
    return make_float2(fmaf(l.t, hr - lr, lr), sgn * fmaf(l.t, hi - li, li));
}

}  // namespace wsp
