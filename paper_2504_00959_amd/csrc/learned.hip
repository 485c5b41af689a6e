// Learned gridding kernel: the paper grids with a Gaussian or Kaiser-Bessel
// kernel (Sec. 2.1, Eq. 3); here a small MLP over (tap offset x, tap offset y,
// w-fraction) is tabulated into a non-separable table indexed by the
// visibility's w-fraction bin, and trained against the direct Fourier sum of
// Eq. 1 through the adjoint of the imaging steps.
//
//   table      T[iw][s_y][s_x][t_y][t_x] = K(dx, dy, f_iw) / sum over the row,
//              K = exp(mlp(dx / (W/2), dy / (W/2), f_iw)) inside |dx|, |dy| < W/2,
//              dx = t_x - h - s_x / OS, f_iw = (iw + 1/2) / N_f - 1/2
//   taper      C(l', m') = (1 / (N_f OS^2)) sum over the table of
//              T cos(2 pi (dx l' + dy m')), as two passes over the W OS
//              distinct offsets per axis (cos(a + b) = cos a cos b - sin a sin b)
//   loss       L = sum_Omega (I - D)^2 / sum_Omega D^2, Omega the inner half of the
//              field; dL/dA = dL/dI / C for the apparent image A = I C and
//              dL/dC = -dL/dI I / C
//   gradient   dL/dG_k is the centred forward DFT of dA n exp(-2 pi i w_k (n - 1)) / sum W
//              (formed as the conjugate of the inverse transform of the
//              conjugate); dL/dT sums Re(dL/dG_k[cell] conj(W V)) over the taps
//              of every visibility, plus the taper's part
//   MLP        3 -> 32 -> 32 -> 1, tanh after the hidden layers, float32;
//              parameters packed W1 [32][3], b1 [32], W2 [32][32], b2 [32],
//              w3 [32], b3
//   direct sum D = n Re(sum_v W V exp(+2 pi i (u l + v m + w (n - 1)))) / sum W over
//              the visibilities the plan keeps, float64 phase and accumulation,
//              float32 sin/cos of the reduced phase
#include <cmath>

#include "rick_internal.h"
#include "quant.h"

namespace rick {

namespace {

constexpr int kHid = 32;
constexpr int kNParam = kHid * 3 + kHid + kHid * kHid + kHid + kHid + 1;   // 1217
constexpr int kBlock = 256;

template <typename real>
struct C2;
template <>
struct C2<float> {
    using t = float2;
};
template <>
struct C2<double> {
    using t = double2;
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// offset of tap t of sub-cell index si (s = si - OS/2): t - h - s / OS
__device__ __forceinline__ double tap_offset(int t, int si, int W, int OS) {
    return (double)(t - (W - 1) / 2) - (double)(si - OS / 2) / (double)OS;
}

// ---- table install: copy (converting to the plan's real type) and the largest |entry| ----
template <typename real>
__global__ __launch_bounds__(kBlock) void k_table_install(const float *__restrict__ src, real *__restrict__ dst,
                                                         int64_t n, unsigned int *__restrict__ tapmax_bits) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const float v = src[i];
        dst[i] = (real)v;
        m = fmaxf(m, fabsf(v));
    }
    // |v| >= 0: the float bit patterns order like the values
    m = fmaxf(m, __shfl_xor(m, 32));
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 8));
    m = fmaxf(m, __shfl_xor(m, 4));
    m = fmaxf(m, __shfl_xor(m, 2));
    m = fmaxf(m, __shfl_xor(m, 1));
    if ((threadIdx.x & 63) == 0) atomicMax(tapmax_bits, __float_as_uint(m));
}

__global__ void k_fill_u32(unsigned int *__restrict__ p, unsigned int v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *__restrict__ p, double v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---- taper ----
// A[y][x] = mean over iw of T[iw][s_y][s_x][t_y][t_x], y = s_y W + t_y, x = s_x W + t_x
template <typename real>
__global__ __launch_bounds__(kBlock) void k_taper_fine(const real *__restrict__ T, int nwf, int OS, int W,
                                                      double *__restrict__ A) {
    const int M = OS * W;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)M * M) return;
    const int y = (int)(i / M), x = (int)(i % M);
    const int sy = y / W, ty = y % W, sx = x / W, tx = x % W;
    double a = 0.0;
    for (int f = 0; f < nwf; ++f) a += (double)T[((((int64_t)f * OS + sy) * OS + sx) * W + ty) * W + tx];
    A[i] = a / nwf;
}

// E_c[j][p] = cos(2 pi d_j l'_p), E_s = sin, d_j = t - h - s/OS (j = s_idx W + t), l'_p = (p - N/2) / N
__global__ __launch_bounds__(kBlock) void k_taper_trig(int OS, int W, int N, double *__restrict__ Ec,
                                                      double *__restrict__ Es) {
    const int M = OS * W;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    const int j = (int)(i / N), p = (int)(i % N);
    const double d = tap_offset(j % W, j / W, W, OS);
    const double lp = (double)(p - N / 2) / (double)N;
    double sn, cs;
    sincospi(2.0 * d * lp, &sn, &cs);
    Ec[i] = cs;
    Es[i] = sn;
}

// out_c[r][p] = sum_j X[r][j] Ec[j][p], out_s likewise (X: [R][M] row-major)
__global__ __launch_bounds__(kBlock) void k_taper_rows(const double *__restrict__ X, const double *__restrict__ Ec,
                                                      const double *__restrict__ Es, int R, int M, int N,
                                                      double *__restrict__ oc, double *__restrict__ os) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)R * N) return;
    const int r = (int)(i / N), p = (int)(i % N);
    double c = 0.0, s = 0.0;
    for (int j = 0; j < M; ++j) {
        const double a = X[(int64_t)r * M + j];
        c = fma(a, Ec[(int64_t)j * N + p], c);
        s = fma(a, Es[(int64_t)j * N + p], s);
    }
    oc[i] = c;
    os[i] = s;
}

// C[q][p] = (1 / OS^2) sum_y (Ec[y][q] Tc[y][p] - Es[y][q] Ts[y][p])
__global__ __launch_bounds__(kBlock) void k_taper_cols(const double *__restrict__ Tc, const double *__restrict__ Ts,
                                                      const double *__restrict__ Ec, const double *__restrict__ Es,
                                                      int M, int N, double inv_os2, double *__restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const int q = (int)(i / N), p = (int)(i % N);
    double c = 0.0;
    for (int y = 0; y < M; ++y) {
        c = fma(Ec[(int64_t)y * N + q], Tc[(int64_t)y * N + p], c);
        c = fma(-Es[(int64_t)y * N + q], Ts[(int64_t)y * N + p], c);
    }
    C[i] = c * inv_os2;
}

// taper adjoint, first pass: U_c[y][p] = sum_q Ec[y][q] dC[q][p], U_s likewise
__global__ __launch_bounds__(kBlock) void k_taper_adj1(const double *__restrict__ dC, const double *__restrict__ Ec,
                                                      const double *__restrict__ Es, int M, int N,
                                                      double *__restrict__ Uc, double *__restrict__ Us) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)M * N) return;
    const int y = (int)(i / N), p = (int)(i % N);
    double c = 0.0, s = 0.0;
    for (int q = 0; q < N; ++q) {
        const double d = dC[(int64_t)q * N + p];
        c = fma(Ec[(int64_t)y * N + q], d, c);
        s = fma(Es[(int64_t)y * N + q], d, s);
    }
    Uc[i] = c;
    Us[i] = s;
}

// second pass: dA[y][x] = (1 / OS^2) sum_p (Uc[y][p] Ec[x][p] - Us[y][p] Es[x][p]);
// every w-fraction bin's entry gets dA / N_f added
template <typename real>
__global__ __launch_bounds__(kBlock) void k_taper_adj2(const double *__restrict__ Uc, const double *__restrict__ Us,
                                                      const double *__restrict__ Ec, const double *__restrict__ Es,
                                                      int nwf, int OS, int W, int N, double inv_os2,
                                                      double *__restrict__ dT) {
    const int M = OS * W;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)M * M) return;
    const int y = (int)(i / M), x = (int)(i % M);
    double a = 0.0;
    for (int p = 0; p < N; ++p) {
        a = fma(Uc[(int64_t)y * N + p], Ec[(int64_t)x * N + p], a);
        a = fma(-Us[(int64_t)y * N + p], Es[(int64_t)x * N + p], a);
    }
    a *= inv_os2 / nwf;
    const int sy = y / W, ty = y % W, sx = x / W, tx = x % W;
    for (int f = 0; f < nwf; ++f) dT[((((int64_t)f * OS + sy) * OS + sx) * W + ty) * W + tx] += a;
}

// ---- loss ----
__device__ __forceinline__ bool in_omega(int q, int p, int N) {
    const int dq = q - N / 2, dp = p - N / 2;
    return (dq < 0 ? -dq : dq) < N / 4 && (dp < 0 ? -dp : dp) < N / 4;
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_loss_sums(const real *__restrict__ I, const double *__restrict__ D, int N,
                                                     double *__restrict__ sums) {
    double a = 0.0, b = 0.0;
    const int64_t n = (int64_t)N * N;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int q = (int)(i / N), p = (int)(i % N);
        if (in_omega(q, p, N)) {
            const double d = (double)I[i] - D[i];
            a = fma(d, d, a);
            b = fma(D[i], D[i], b);
        }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sums[0], a);
        atomicAdd(&sums[1], b);
    }
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_loss_grad(Geom g, const real *__restrict__ I, const double *__restrict__ D,
                                                     const double *__restrict__ taper, const double *__restrict__ sums,
                                                     double *__restrict__ dA, double *__restrict__ dC) {
    const int N = g.N;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const int q = (int)(i / N), p = (int)(i % N);
    const double den = sums[1];
    double a = 0.0, c = 0.0;
    if (in_omega(q, p, N) && den > 0.0) {
        const double cc = taper_at(g, taper, q, p);
        const double dI = 2.0 * ((double)I[i] - D[i]) / den;
        a = dI / cc;
        c = -dI * (double)I[i] / cc;
    }
    dA[i] = a;
    dC[i] = c;
}

// ---- table gradient ----
// conj(dL/dG_k) planes before the inverse FFT: conj of dA n exp(-2 pi i w_k (n - 1)) / sum W
template <typename real>
__global__ __launch_bounds__(kBlock) void k_grad_screen(Geom g, const double *__restrict__ dA,
                                                       const Stats *__restrict__ st, real *__restrict__ mesh) {
    using C = typename C2<real>::t;
    const int64_t npix = (int64_t)g.N * g.N;
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    const int q = (int)(pix / g.N), p = (int)(pix % g.N);
    const double dl = g.fov / g.N;
    const double l = (double)(p - g.N / 2) * dl, m = (double)(q - g.N / 2) * dl;
    const double r2 = l * l + m * m;
    const bool inside = r2 < 1.0;
    const double nm1 = inside ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
    const double sw = st->sum_w;
    const double base = (inside && sw > 0.0) ? dA[pix] * (1.0 + nm1) / sw : 0.0;
    C *out = reinterpret_cast<C *>(mesh) + pix;
    for (int k = 0; k < g.Nw; ++k) {
        const double tau = plane_centre(g, k) * nm1;
        double sn, cs;
        sincospi(2.0 * (tau - rint(tau)), &sn, &cs);
        C v;
        v.x = (real)(base * cs);   // conj(exp(-2 pi i tau)) = exp(+2 pi i tau)
        v.y = (real)(base * sn);
        out[(int64_t)k * npix] = v;
    }
}

// dL/dT[iw][s_y][s_x][t_y][t_x] += Re(dL/dG_k[cell] conj(W V)) = Re(H[cell] W V)
// with H = conj(dL/dG_k) in the mesh; one thread per visibility
template <typename real>
__global__ __launch_bounds__(kBlock) void k_table_grad(Geom g, const double *__restrict__ uvw,
                                                      const double *__restrict__ scales, const real *__restrict__ vis,
                                                      const float *__restrict__ weight, int64_t nrow, int32_t nchan,
                                                      const real *__restrict__ mesh, double *__restrict__ dT) {
#pragma clang fp contract(off)
    using C = typename C2<real>::t;
    const int64_t nvis = nrow * nchan;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nvis) return;
    const int64_t r = i / nchan;
    const int32_t c = (int32_t)(i - r * nchan);
    const double sc = scales[c];
    const double u = uvw[3 * r] * sc, v = uvw[3 * r + 1] * sc, w = uvw[3 * r + 2] * sc;
    const real vr = vis[2 * i], vi = vis[2 * i + 1];
    const float wt = weight ? weight[i] : 1.0f;
    Quant qd;
    if (!quantise(g, u, v, w, vr, vi, wt, qd)) return;
    const double ar = (double)wt * (double)vr, ai = (double)wt * (double)vi;
    const int W = g.W;
    const int64_t row = (((int64_t)qd.iw * g.OS + qd.sy + g.OS / 2) * g.OS + qd.sx + g.OS / 2) * W * W;
    const C *plane = reinterpret_cast<const C *>(mesh) + (int64_t)qd.k * g.N * g.N;
    for (int ty = 0; ty < W; ++ty) {
        const C *line = plane + (int64_t)(qd.cy + ty - g.h) * g.N + (qd.cx - g.h);
        for (int tx = 0; tx < W; ++tx) {
            const C h = line[tx];
            atomicAdd(&dT[row + ty * W + tx], (double)h.x * ar - (double)h.y * ai);
        }
    }
}

// ---- MLP ----
struct MlpOut {
    float y;
    float a1[kHid], a2[kHid];
};

__device__ __forceinline__ void mlp_eval(const float *__restrict__ th, float x0, float x1, float x2, MlpOut &o) {
    const float *W1 = th, *b1 = W1 + kHid * 3, *W2 = b1 + kHid, *b2 = W2 + kHid * kHid, *w3 = b2 + kHid;
    const float b3 = w3[kHid];
#pragma unroll
    for (int j = 0; j < kHid; ++j) o.a1[j] = tanhf(fmaf(W1[3 * j + 2], x2, fmaf(W1[3 * j + 1], x1, fmaf(W1[3 * j], x0, b1[j]))));
    float y = b3;
#pragma unroll 4
    for (int i = 0; i < kHid; ++i) {
        float z = b2[i];
#pragma unroll
        for (int j = 0; j < kHid; ++j) z = fmaf(W2[kHid * i + j], o.a1[j], z);
        o.a2[i] = tanhf(z);
        y = fmaf(w3[i], o.a2[i], y);
    }
    o.y = y;
}

// one wave per table row (iw, s_y, s_x); W^2 taps over the lanes (in turns for W > 7)
constexpr int kMaxTapsPerLane = 4;   // W <= 15: 225 taps
__global__ __launch_bounds__(kBlock) void k_mlp_table(const float *__restrict__ theta, int W, int OS, int nwf,
                                                     float *__restrict__ T, float *__restrict__ rowsum) {
    __shared__ float s_th[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += kBlock) s_th[i] = theta[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nrows = (int64_t)nwf * OS * OS;
    if (row >= nrows) return;
    const int f = (int)(row / ((int64_t)OS * OS)), sy = (int)((row / OS) % OS), sx = (int)(row % OS);
    const int W2 = W * W;
    const double half = W / 2.0;
    const float fw = (float)(((double)f + 0.5) / (double)nwf - 0.5);
    float K[kMaxTapsPerLane];
    float sum = 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxTapsPerLane; ++j) {
        const int t = lane + 64 * j;
        K[j] = 0.0f;
        if (t < W2) {
            const double dx = tap_offset(t % W, sx, W, OS), dy = tap_offset(t / W, sy, W, OS);
            if (fabs(dx) < half && fabs(dy) < half) {
                MlpOut o;
                mlp_eval(s_th, (float)(dx / half), (float)(dy / half), fw, o);
                K[j] = expf(o.y);
            }
        }
        sum += K[j];
    }
    sum = wave_sum(sum);
#pragma unroll
    for (int j = 0; j < kMaxTapsPerLane; ++j) {
        const int t = lane + 64 * j;
        if (t < W2) T[row * W2 + t] = K[j] / sum;
    }
    if (lane == 0 && rowsum) rowsum[row] = sum;
}

// Parameter gradient of sum(dT T).  T = K / S (S the row sum), K = exp(y):
// dy = (dT - sum_row(dT T)) T.  One wave per table row: the per-tap factors
// of the backward pass are staged in LDS and reduced per parameter, and each
// wave adds its sums to the gradient.
constexpr int kBwd = 64;
__global__ __launch_bounds__(kBwd) void k_mlp_backward(const float *__restrict__ theta, int W, int OS, int nwf,
                                                      const float *__restrict__ T, const double *__restrict__ dT,
                                                      float *__restrict__ dtheta) {
    __shared__ float s_th[kNParam];
    __shared__ float s_d2[kBwd][kHid + 1];   // dz2 of every lane's tap
    __shared__ float s_a1[kBwd][kHid + 1];   // a1
    __shared__ float s_d1[kBwd][kHid + 1];   // dz1
    __shared__ float s_a2[kBwd][kHid + 1];   // a2
    __shared__ float s_x[kBwd][4];           // inputs and dy
    for (int i = threadIdx.x; i < kNParam; i += kBwd) s_th[i] = theta[i];
    __syncthreads();
    const float *W2 = s_th + kHid * 4, *w3 = W2 + kHid * kHid + kHid;
    const int lane = threadIdx.x;
    const int W2n = W * W;
    const int64_t row = blockIdx.x;
    const double half = W / 2.0;
    const int f = (int)(row / ((int64_t)OS * OS)), sy = (int)((row / OS) % OS), sx = (int)(row % OS);
    double sdt = 0.0;
    for (int j = lane; j < W2n; j += kBwd) sdt += dT[row * W2n + j] * (double)T[row * W2n + j];
    sdt = wave_sum(sdt);
    float grad[(kNParam + kBwd - 1) / kBwd];
#pragma unroll
    for (int a = 0; a < (kNParam + kBwd - 1) / kBwd; ++a) grad[a] = 0.0f;
    for (int part = 0; part < kMaxTapsPerLane && 64 * part < W2n; ++part) {
        const int t = lane + 64 * part;
        float dy = 0.0f, x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
        MlpOut o;
        bool on = false;
        if (t < W2n) {
            const double dx = tap_offset(t % W, sx, W, OS), dyo = tap_offset(t / W, sy, W, OS);
            if (fabs(dx) < half && fabs(dyo) < half) {
                on = true;
                x0 = (float)(dx / half);
                x1 = (float)(dyo / half);
                x2 = (float)(((double)f + 0.5) / (double)nwf - 0.5);
                dy = (float)((dT[row * W2n + t] - sdt) * (double)T[row * W2n + t]);
            }
        }
        if (on) mlp_eval(s_th, x0, x1, x2, o);
#pragma unroll
        for (int i = 0; i < kHid; ++i) {
            const float a2 = on ? o.a2[i] : 0.0f;
            s_a2[lane][i] = a2;
            s_d2[lane][i] = on ? dy * w3[i] * (1.0f - a2 * a2) : 0.0f;
            s_a1[lane][i] = on ? o.a1[i] : 0.0f;
        }
#pragma unroll 4
        for (int j = 0; j < kHid; ++j) {
            float sacc = 0.0f;
#pragma unroll
            for (int i = 0; i < kHid; ++i) sacc = fmaf(s_d2[lane][i], W2[kHid * i + j], sacc);
            s_d1[lane][j] = on ? sacc * (1.0f - s_a1[lane][j] * s_a1[lane][j]) : 0.0f;
        }
        s_x[lane][0] = x0;
        s_x[lane][1] = x1;
        s_x[lane][2] = x2;
        s_x[lane][3] = on ? dy : 0.0f;
        __syncthreads();
        // lane owns parameters lane, lane + 64, ...; sums over the row's taps
#pragma unroll
        for (int a = 0; a < (kNParam + kBwd - 1) / kBwd; ++a) {
            const int pidx = lane + kBwd * a;
            float g = 0.0f;
            if (pidx < kHid * 3) {                                   // W1[j][c]
                const int j = pidx / 3, c = pidx % 3;
                for (int e = 0; e < kBwd; ++e) g = fmaf(s_d1[e][j], s_x[e][c], g);
            } else if (pidx < kHid * 4) {                            // b1[j]
                const int j = pidx - kHid * 3;
                for (int e = 0; e < kBwd; ++e) g += s_d1[e][j];
            } else if (pidx < kHid * 4 + kHid * kHid) {              // W2[i][j]
                const int q = pidx - kHid * 4, i = q / kHid, j = q % kHid;
                for (int e = 0; e < kBwd; ++e) g = fmaf(s_d2[e][i], s_a1[e][j], g);
            } else if (pidx < kHid * 5 + kHid * kHid) {              // b2[i]
                const int i = pidx - kHid * 4 - kHid * kHid;
                for (int e = 0; e < kBwd; ++e) g += s_d2[e][i];
            } else if (pidx < kHid * 6 + kHid * kHid) {              // w3[i]
                const int i = pidx - kHid * 5 - kHid * kHid;
                for (int e = 0; e < kBwd; ++e) g = fmaf(s_x[e][3], s_a2[e][i], g);
            } else if (pidx < kNParam) {                             // b3
                for (int e = 0; e < kBwd; ++e) g += s_x[e][3];
            }
            grad[a] += g;
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < (kNParam + kBwd - 1) / kBwd; ++a) {
        const int pidx = lane + kBwd * a;
        if (pidx < kNParam && grad[a] != 0.0f) atomicAdd(&dtheta[pidx], grad[a]);
    }
}

// Adam (Kingma & Ba 2015, Algorithm 1): m = b1 m + (1 - b1) g,
// v = b2 v + (1 - b2) g^2, theta -= lr m_hat / (sqrt(v_hat) + eps) with
// m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t) (c1, c2 the two reciprocals)
__global__ void k_adam(float *__restrict__ th, const float *__restrict__ gr, float *__restrict__ m,
                       float *__restrict__ v, int n, float b1, float b2, float lr, float c1, float c2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ---- a separable table in the non-separable layout, and a table residual ----
// out[iw][s_y][s_x][t_y][t_x] = g[s_y][t_y] g[s_x][t_x] (g the plan's separable rows)
template <typename real>
__global__ __launch_bounds__(kBlock) void k_separable_table(const real *__restrict__ g, int nwf, int OS, int W,
                                                           float *__restrict__ out) {
    const int64_t n = (int64_t)nwf * OS * OS * W * W;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int tx = (int)(i % W), ty = (int)((i / W) % W);
    const int sx = (int)((i / (W * W)) % OS), sy = (int)((i / ((int64_t)W * W * OS)) % OS);
    out[i] = (float)((double)g[sy * W + ty] * (double)g[sx * W + tx]);
}

// dT = 2 (T - R) / n and sums[0] = sum (T - R)^2 / n (a least-squares fit of a table to R)
__global__ __launch_bounds__(kBlock) void k_table_residual(const float *__restrict__ T, const float *__restrict__ R,
                                                          int64_t n, double *__restrict__ dT,
                                                          double *__restrict__ sums) {
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double d = (double)T[i] - (double)R[i];
        dT[i] = 2.0 * d / (double)n;
        a = fma(d, d, a);
    }
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) atomicAdd(&sums[0], a / (double)n);
}

// ---- direct Fourier sum at a rectangle of pixels ----
constexpr int kDftPix = 256;      // pixels per block (one per thread)
constexpr int kDftVis = 16384;    // visibilities per block
constexpr int kDftStage = 256;    // visibilities staged in LDS at a time
template <typename real>
__global__ __launch_bounds__(kBlock) void k_dft(Geom g, const double *__restrict__ uvw,
                                               const double *__restrict__ scales, const real *__restrict__ vis,
                                               const float *__restrict__ weight, int64_t nrow, int32_t nchan,
                                               int q0, int p0, int nq, int np, double *__restrict__ out,
                                               double *__restrict__ wsum) {
#pragma clang fp contract(off)
    __shared__ double s_u[kDftStage], s_v[kDftStage], s_w[kDftStage], s_ar[kDftStage], s_ai[kDftStage];
    const int64_t npix = (int64_t)nq * np;
    const int64_t pix = (int64_t)blockIdx.x * kDftPix + threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.y * kDftVis;
    const int64_t nvis = nrow * nchan;
    const bool have = pix < npix;
    const int q = have ? q0 + (int)(pix / np) : 0, p = have ? p0 + (int)(pix % np) : 0;
    const double dl = g.fov / g.N;
    const double l = (double)(p - g.N / 2) * dl, m = (double)(q - g.N / 2) * dl;
    const double r2 = l * l + m * m;
    const double nm1 = r2 < 1.0 ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
    double acc = 0.0, ws = 0.0;
    for (int64_t s0 = v0; s0 < v0 + kDftVis && s0 < nvis; s0 += kDftStage) {
        __syncthreads();
        {
            const int64_t i = s0 + threadIdx.x;
            double u = 0, v = 0, w = 0, ar = 0, ai = 0;
            if (i < nvis && i < v0 + kDftVis) {
                const int64_t r = i / nchan;
                const int32_t c = (int32_t)(i - r * nchan);
                const double sc = scales[c];
                u = uvw[3 * r] * sc;
                v = uvw[3 * r + 1] * sc;
                w = uvw[3 * r + 2] * sc;
                const real vr = vis[2 * i], vi = vis[2 * i + 1];
                const float wt = weight ? weight[i] : 1.0f;
                Quant qd;
                if (quantise(g, u, v, w, vr, vi, wt, qd)) {
                    ar = (double)wt * (double)vr;
                    ai = (double)wt * (double)vi;
                    ws += (double)wt;
                }
            }
            s_u[threadIdx.x] = u;
            s_v[threadIdx.x] = v;
            s_w[threadIdx.x] = w;
            s_ar[threadIdx.x] = ar;
            s_ai[threadIdx.x] = ai;
        }
        __syncthreads();
        if (have) {
            for (int j = 0; j < kDftStage; ++j) {
                // phase in float64 half turns, nearest integer out, float32 sin/cos of the rest
                const double t2 = 2.0 * (s_u[j] * l + s_v[j] * m + s_w[j] * nm1);
                const double qd = rint(t2);
                float sn, cs;
                sincospi_half((float)(t2 - qd), sn, cs);
                const double sg = ((long long)qd & 1) ? -1.0 : 1.0;
                acc = fma(sg * s_ar[j], (double)cs, acc);
                acc = fma(-sg * s_ai[j], (double)sn, acc);
            }
        }
    }
    if (have) atomicAdd(&out[pix], acc);
    // the weight sum: once per visibility (blocks of the first pixel tile only)
    if (blockIdx.x == 0) {
        ws = wave_sum(ws);
        if ((threadIdx.x & 63) == 0) atomicAdd(wsum, ws);
    }
}

__global__ __launch_bounds__(kBlock) void k_dft_finish(Geom g, int q0, int p0, int nq, int np,
                                                      const double *__restrict__ wsum, double *__restrict__ out) {
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= (int64_t)nq * np) return;
    const int q = q0 + (int)(pix / np), p = p0 + (int)(pix % np);
    const double dl = g.fov / g.N;
    const double l = (double)(p - g.N / 2) * dl, m = (double)(q - g.N / 2) * dl;
    const double r2 = l * l + m * m;
    const double sw = *wsum;
    if (!(r2 < 1.0) || !(sw > 0.0)) {
        out[pix] = 0.0;
        return;
    }
    const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
    out[pix] = (1.0 + nm1) * out[pix] / sw;
}

unsigned blocks_for(int64_t n, int per = kBlock, int64_t cap = 1 << 20) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    return (unsigned)(b < cap ? b : cap);
}

}  // namespace

int mlp_param_count() { return kNParam; }

template <typename real>
hipError_t launch_table_install(const float *src, real *dst, int64_t n, float *tapmax, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned int *>(tapmax), 0u, (int64_t)1);
    hipLaunchKernelGGL((k_table_install<real>), dim3(blocks_for(n, kBlock, 4096)), dim3(kBlock), 0, s, src, dst, n,
                       reinterpret_cast<unsigned int *>(tapmax));
    return hipGetLastError();
}

template <typename real>
hipError_t launch_taper2d(const Geom &g, const real *T, const TaperBufs &tb, double *C, hipStream_t s) {
    const int M = g.OS * g.W, N = g.N;
    hipLaunchKernelGGL((k_taper_fine<real>), dim3(blocks_for((int64_t)M * M)), dim3(kBlock), 0, s, T, g.nwf, g.OS,
                       g.W, tb.A);
    hipLaunchKernelGGL(k_taper_trig, dim3(blocks_for((int64_t)M * N)), dim3(kBlock), 0, s, g.OS, g.W, N, tb.Ec, tb.Es);
    hipLaunchKernelGGL(k_taper_rows, dim3(blocks_for((int64_t)M * N)), dim3(kBlock), 0, s, tb.A, tb.Ec, tb.Es, M, M,
                       N, tb.Uc, tb.Us);
    hipLaunchKernelGGL(k_taper_cols, dim3(blocks_for((int64_t)N * N)), dim3(kBlock), 0, s, tb.Uc, tb.Us, tb.Ec, tb.Es,
                       M, N, 1.0 / ((double)g.OS * g.OS), C);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_taper2d_adjoint(const Geom &g, const double *dC, const TaperBufs &tb, double *dT, hipStream_t s) {
    const int M = g.OS * g.W, N = g.N;
    hipLaunchKernelGGL(k_taper_adj1, dim3(blocks_for((int64_t)M * N)), dim3(kBlock), 0, s, dC, tb.Ec, tb.Es, M, N,
                       tb.Uc, tb.Us);
    hipLaunchKernelGGL((k_taper_adj2<real>), dim3(blocks_for((int64_t)M * M)), dim3(kBlock), 0, s, tb.Uc, tb.Us,
                       tb.Ec, tb.Es, g.nwf, g.OS, g.W, N, 1.0 / ((double)g.OS * g.OS), dT);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_image_loss(const Geom &g, const real *I, const double *D, const double *taper, double *dA,
                             double *dC, double *sums, hipStream_t s) {
    const int64_t n = (int64_t)g.N * g.N;
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, sums, 0.0, (int64_t)2);
    hipLaunchKernelGGL((k_loss_sums<real>), dim3(blocks_for(n, kBlock, 2048)), dim3(kBlock), 0, s, I, D, g.N, sums);
    hipLaunchKernelGGL((k_loss_grad<real>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, I, D, taper, sums, dA, dC);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_grad_screen(const Geom &g, const double *dA, const Stats *st, real *mesh, hipStream_t s) {
    hipLaunchKernelGGL((k_grad_screen<real>), dim3(blocks_for((int64_t)g.N * g.N)), dim3(kBlock), 0, s, g, dA, st,
                       mesh);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_table_grad(const Geom &g, const double *uvw, const double *scales, const real *vis,
                             const float *weight, int64_t nrow, int32_t nchan, const real *mesh, double *dT,
                             int64_t n_table, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n_table, kBlock, 4096)), dim3(kBlock), 0, s, dT, 0.0, n_table);
    hipLaunchKernelGGL((k_table_grad<real>), dim3(blocks_for(nrow * nchan)), dim3(kBlock), 0, s, g, uvw, scales, vis,
                       weight, nrow, nchan, mesh, dT);
    return hipGetLastError();
}

hipError_t launch_mlp_table(const float *theta, int W, int OS, int nwf, float *T, float *rowsum, hipStream_t s) {
    const int64_t nrows = (int64_t)nwf * OS * OS;
    hipLaunchKernelGGL(k_mlp_table, dim3(blocks_for(nrows, kBlock / 64)), dim3(kBlock), 0, s, theta, W, OS, nwf, T,
                       rowsum);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *theta, int W, int OS, int nwf, const float *T, const double *dT,
                               float *dtheta, hipStream_t s) {
    const int64_t nrows = (int64_t)nwf * OS * OS;
    hipLaunchKernelGGL(k_fill_u32, dim3(8), dim3(256), 0, s, reinterpret_cast<unsigned int *>(dtheta), 0u,
                       (int64_t)kNParam);
    hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)nrows), dim3(kBwd), 0, s, theta, W, OS, nwf, T, dT, dtheta);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, theta, grad, m, v, n, b1, b2, lr, c1, c2, eps);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_dft(const Geom &g, const double *uvw, const double *scales, const real *vis, const float *weight,
                      int64_t nrow, int32_t nchan, int q0, int p0, int nq, int np, double *out, double *wsum,
                      hipStream_t s) {
    const int64_t npix = (int64_t)nq * np, nvis = nrow * nchan;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(npix, kBlock, 4096)), dim3(kBlock), 0, s, out, 0.0, npix);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, wsum, 0.0, (int64_t)1);
    const int64_t gy = (nvis + kDftVis - 1) / kDftVis;
    if (gy > 65535) return hipErrorInvalidValue;
    if (nvis > 0) {
        dim3 grid((unsigned)((npix + kDftPix - 1) / kDftPix), (unsigned)gy);
        hipLaunchKernelGGL((k_dft<real>), grid, dim3(kBlock), 0, s, g, uvw, scales, vis, weight, nrow, nchan, q0, p0,
                           nq, np, out, wsum);
    }
    hipLaunchKernelGGL(k_dft_finish, dim3(blocks_for(npix)), dim3(kBlock), 0, s, g, q0, p0, nq, np, wsum, out);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_separable_table(const real *g, int nwf, int OS, int W, float *out, hipStream_t s) {
    const int64_t n = (int64_t)nwf * OS * OS * W * W;
    hipLaunchKernelGGL((k_separable_table<real>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, nwf, OS, W, out);
    return hipGetLastError();
}

hipError_t launch_table_residual(const float *T, const float *R, int64_t n, double *dT, double *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, sums, 0.0, (int64_t)1);
    hipLaunchKernelGGL(k_table_residual, dim3(blocks_for(n, kBlock, 2048)), dim3(kBlock), 0, s, T, R, n, dT, sums);
    return hipGetLastError();
}

#define INST(real)                                                                                                  \
    template hipError_t launch_separable_table<real>(const real *, int, int, int, float *, hipStream_t);           \
    template hipError_t launch_table_install<real>(const float *, real *, int64_t, float *, hipStream_t);            \
    template hipError_t launch_taper2d<real>(const Geom &, const real *, const TaperBufs &, double *, hipStream_t);   \
    template hipError_t launch_taper2d_adjoint<real>(const Geom &, const double *, const TaperBufs &, double *,       \
                                                     hipStream_t);                                                   \
    template hipError_t launch_image_loss<real>(const Geom &, const real *, const double *, const double *, double *, \
                                                double *, double *, hipStream_t);                                    \
    template hipError_t launch_grad_screen<real>(const Geom &, const double *, const Stats *, real *, hipStream_t);   \
    template hipError_t launch_table_grad<real>(const Geom &, const double *, const double *, const real *,          \
                                                const float *, int64_t, int32_t, const real *, double *, int64_t,    \
                                                hipStream_t);                                                        \
    template hipError_t launch_dft<real>(const Geom &, const double *, const double *, const real *, const float *,   \
                                         int64_t, int32_t, int, int, int, int, double *, double *, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace rick
