/* Per-visibility position, plane and drop decision of the oracle --
 * TEST INFRASTRUCTURE ONLY.  The same float64 steps, in the same order, as
 * oracle/wstack.py bin_visibilities (Sec. 2.1: closest w-plane, 1/OS
 * quantised position, nearest cell).  Used by the oracle's C passes only. */
#ifndef ORACLE_DECIDE_H
#define ORACLE_DECIDE_H
#include <math.h>
#include <stdint.h>

static inline int64_t oracle_floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

typedef struct {
    int64_t cx, cy, sx, sy, k;
    double wt, ar, ai;   /* weight and W * V */
} oracle_vis_t;

/* Returns 1 if visibility (r, c) is kept, filling *o. */
static inline int oracle_decide(int64_t r, int32_t c, int32_t nchan, const double *uvw, const double *scales,
                                const float *vis, const float *weight, int64_t N, int64_t OS, int64_t h,
                                int32_t nw, double fov, double w_min, double dw, oracle_vis_t *o)
{
    double u, v, w;
    if (scales) {
        u = uvw[3 * r] * scales[c];
        v = uvw[3 * r + 1] * scales[c];
        w = uvw[3 * r + 2] * scales[c];
    } else {
        u = uvw[3 * r]; v = uvw[3 * r + 1]; w = uvw[3 * r + 2];
    }
    const int64_t vi = r * nchan + c;
    const double vr = vis[2 * vi], vim = vis[2 * vi + 1];
    const double wt = weight ? (double)weight[vi] : 1.0;
    if (!(isfinite(u) && isfinite(v) && isfinite(w) && isfinite(vr) && isfinite(vim) && isfinite(wt)))
        return 0;
    const double half = (double)(N * OS) / 2.0;
    double xs = u * fov; xs = xs * (double)OS; xs = xs + half;
    double ys = v * fov; ys = ys * (double)OS; ys = ys + half;
    if (!(fabs(xs) <= 1073741824.0 && fabs(ys) <= 1073741824.0)) return 0;
    const int64_t X = (int64_t)rint(xs), Y = (int64_t)rint(ys);
    o->cx = oracle_floordiv(X + OS / 2, OS);
    o->cy = oracle_floordiv(Y + OS / 2, OS);
    o->sx = X - o->cx * OS;
    o->sy = Y - o->cy * OS;
    if (!(wt > 0.0)) return 0;
    if (o->cx - h < 0 || o->cx + h > N - 1 || o->cy - h < 0 || o->cy + h > N - 1) return 0;
    double kf = floor((w - w_min) / dw);
    if (isnan(kf)) kf = 0.0;   /* w outside the range -> nearest end plane */
    if (kf < 0.0) kf = 0.0;
    if (kf > (double)(nw - 1)) kf = (double)(nw - 1);
    o->k = (int64_t)kf;
    o->wt = wt;
    o->ar = wt * vr;
    o->ai = wt * vim;
    return 1;
}
#endif
