// Position quantisation, closest w-plane and drop decision of one
// visibility (Sec. 2.1): shared by binning (imaging) and by interpolation
// (prediction), so that both directions place a visibility identically.
//   X = rint((u FoV) OS + N OS / 2), c_x = floor((X + OS/2) / OS), s_x = X - c_x OS
//   k = clamp(floor((w - w_min) / dw), 0, N_w - 1)
//   with a non-separable table of N_f w-fraction bins:
//   iw = clamp(floor(((w - w_min) / dw - k) N_f), 0, N_f - 1)
//   dropped if any input is non-finite, the position is beyond 2^30
//   sub-cells, the weight is <= 0, or the W x W footprint leaves the grid.
// quantise_pos takes every decision but the finiteness of V, so that the
// binning's counting pass need not read the visibilities.
#pragma once
#include "rick_internal.h"

namespace rick {

struct Quant {
    int32_t cx, cy, sx, sy, k;
    int32_t iw;   // w-fraction bin (0 with a separable tap table)
};

// Position, plane and drop decision of one visibility from (u, v, w) and its
// weight alone (every test but the finiteness of V), evaluated without
// branches (every lane computes every step; the decisions are combined at
// the end), which keeps the loop free of execution-mask changes.
__device__ __forceinline__ bool quantise_pos(const Geom &g, double u, double v, double w, float wt, Quant &q) {
#pragma clang fp contract(off)
    // (bitwise & on 0/1 integers on purpose: no short-circuit branches)
    unsigned ok = (unsigned)isfinite(u) & (unsigned)isfinite(v) & (unsigned)isfinite(w) & (unsigned)isfinite(wt);
    double xs = u * g.fov;
    xs = xs * (double)g.OS;
    xs = xs + g.half;
    double ys = v * g.fov;
    ys = ys * (double)g.OS;
    ys = ys + g.half;
    ok &= (unsigned)(fabs(xs) <= 1073741824.0) & (unsigned)(fabs(ys) <= 1073741824.0);
    const int32_t X = ok ? (int32_t)rint(xs) : 0;
    const int32_t Y = ok ? (int32_t)rint(ys) : 0;
    q.cx = (X + (g.OS >> 1)) >> g.log2OS;   // floor division by OS (arithmetic shift)
    q.cy = (Y + (g.OS >> 1)) >> g.log2OS;
    q.sx = X - (q.cx << g.log2OS);
    q.sy = Y - (q.cy << g.log2OS);
    ok &= (unsigned)(wt > 0.0f);
    ok &= (unsigned)(q.cx - g.h >= 0) & (unsigned)(q.cx + g.h <= g.N - 1) & (unsigned)(q.cy - g.h >= 0) &
          (unsigned)(q.cy + g.h <= g.N - 1);
    const double rw = (w - g.w_min) / g.dw;
    double kf = floor(rw);
    if (isnan(kf)) kf = 0.0;
    kf = kf < 0.0 ? 0.0 : kf;
    kf = kf > (double)(g.Nw - 1) ? (double)(g.Nw - 1) : kf;
    q.k = (int32_t)kf;
    // w-fraction bin of a non-separable table: floor((r - k) N_f), clamped
    // (r - k leaves [0, 1) only for w outside the planes' range)
    q.iw = 0;
    if (g.nwf > 1) {
        double fb = floor((rw - kf) * (double)g.nwf);
        if (!isfinite(fb)) fb = 0.0;
        fb = fb < 0.0 ? 0.0 : fb;
        fb = fb > (double)(g.nwf - 1) ? (double)(g.nwf - 1) : fb;
        q.iw = (int32_t)fb;
    }
    if (!ok) q = Quant{0, 0, 0, 0, 0, 0};
    return ok != 0u;
}

// The whole decision: quantise_pos and a finite V.
template <typename real>
__device__ __forceinline__ bool quantise(const Geom &g, double u, double v, double w, real vr, real vi, float wt,
                                         Quant &q) {
    const bool ok = quantise_pos(g, u, v, w, wt, q) & isfinite((double)vr) & isfinite((double)vi);
    if (!ok) q = Quant{0, 0, 0, 0, 0, 0};
    return ok;
}

}  // namespace rick
