// DeepFlow (Sec. 4.3): variational refinement of a flow field with
// DeepMatching's matches as the matching term, coarse to fine.
//
// Energy (Eq. (17)): a data term of normalised colour and gradient constancy
// (Eq. (18)), a smoothness term weighted by alpha(x) = exp(-kappa |grad I|)
// (Eq. (19)) and c phi Psi(|w - w'|^2), every term penalised by
// Psi(s^2) = sqrt(s^2 + eps^2).  At each level of the eta-pyramid the second
// image is warped by the current flow, the constancy assumptions are
// linearised in the increment (du, dv), and a few fixed-point iterations
// freeze the penalisers' derivatives so that the increment solves a linear
// system: a 2 x 2 block per pixel, coupled to the 4 neighbours through the
// smoothness weights, solved by red-black block SOR.  The matching weight at
// level k is beta (k / k_max)^b.
//
// Every step is an elementwise or 3 x 3-stencil pass over one level's maps
// (a few MB at most): the kernels are bandwidth- and launch-bound, one thread
// per pixel, coalesced along rows.  All maps are FP32, row-major, one array
// per quantity (structure of arrays), in the caller's workspace.
//
// Discretisation choices where the paper leaves them open (images in [0, 1]
// for the data and smoothness terms, 0..255 for phi; level sizes
// round(W eta^k) down to a smaller side of min_size; bilinear resampling with
// aligned pixel centres; central differences with replicated borders; the
// average of I1 and the warped I2 for spatial derivatives; a 4-neighbour edge
// weighted by the mean of its pixels' alpha psi'; red-black ordering; the
// first match in list order owning a level pixel) are stated in the header.
#include <math.h>
#include <string.h>

#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <vector>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int kDfThreads = 256;
constexpr int kDfMaxRadius = 7;   // Gaussian taps: radius ceil(3 sigma) <= 7

struct Taps {
    float k[2 * kDfMaxRadius + 1];
    int r;
};

inline unsigned nblk(long n) { return (unsigned)((n + kDfThreads - 1) / kDfThreads); }

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ inline float psi_prime(float s2, float eps) { return 0.5f / sqrtf(s2 + eps * eps); }

// Bilinear sample of a w x h map at real (x, y), coordinates clamped to the map.
__device__ inline float bilinear(const float* __restrict__ m, int w, int h, float x, float y) {
    x = fminf(fmaxf(x, 0.f), (float)(w - 1));
    y = fminf(fmaxf(y, 0.f), (float)(h - 1));
    const int x0 = (int)floorf(x), y0 = (int)floorf(y);
    const int x1 = min(x0 + 1, w - 1), y1 = min(y0 + 1, h - 1);
    const float fx = x - (float)x0, fy = y - (float)y0;
    const float top = m[(size_t)y0 * w + x0] * (1.f - fx) + m[(size_t)y0 * w + x1] * fx;
    const float bot = m[(size_t)y1 * w + x0] * (1.f - fx) + m[(size_t)y1 * w + x1] * fx;
    return top * (1.f - fy) + bot * fy;
}

// ---------------------------------------------------------------- image passes
// Separable Gaussian, replicated borders: horizontal pass from the caller's
// image (leading dimension ld), then vertical.
__global__ void k_df_smooth_h(const float* __restrict__ src, int W, int H, int ld, Taps t, float* __restrict__ dst) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= (long)W * H) return;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    float acc = 0.f;
    for (int j = -t.r; j <= t.r; ++j) acc += t.k[j + t.r] * src[(size_t)y * ld + clampi(x + j, 0, W - 1)];
    dst[i] = acc;
}
__global__ void k_df_smooth_v(const float* __restrict__ src, int W, int H, Taps t, float* __restrict__ dst) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= (long)W * H) return;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    float acc = 0.f;
    for (int j = -t.r; j <= t.r; ++j) acc += t.k[j + t.r] * src[(size_t)clampi(y + j, 0, H - 1) * W + x];
    dst[i] = acc;
}

// dst_k (W x H) = mul_k * bilinear resampling of src_k (w x h), pixel
// centres aligned, for the two maps k = 0, 1 (the two images of a pyramid
// level, or the two flow components).
struct Resize2 {
    const float* src[2];
    float* dst[2];
    float mul[2];
};
__global__ void k_df_resize2(Resize2 r, int w, int h, int W, int H) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= (long)W * H) return;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    const float sx = ((float)x + 0.5f) * ((float)w / (float)W) - 0.5f;
    const float sy = ((float)y + 0.5f) * ((float)h / (float)H) - 0.5f;
#pragma unroll
    for (int k = 0; k < 2; ++k) r.dst[k][i] = r.mul[k] * bilinear(r.src[k], w, h, sx, sy);
}

__global__ void k_df_fill2(float* __restrict__ p, float* __restrict__ q, long n, float v) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= n) return;
    p[i] = v;
    q[i] = v;
}
__global__ void k_df_fill_i32(int* __restrict__ p, long n, int v) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- matching term
struct PhiArgs {
    int W, H, max_matches;
    float lam_scale, sigma_m;
};

// Central differences of m at (x, y) with replicated borders.
__device__ inline void grad_at(const float* __restrict__ m, int W, int H, int x, int y, float& gx, float& gy) {
    const float* r = m + (size_t)y * W;
    gx = 0.5f * (r[min(x + 1, W - 1)] - r[max(x - 1, 0)]);
    gy = 0.5f * (m[(size_t)min(y + 1, H - 1) * W + x] - m[(size_t)max(y - 1, 0) * W + x]);
}

// phi of every match on the smoothed full-size images, read on 0..255
// intensities: sqrt(lambda~) / (sigma_M sqrt(2 pi)) exp(-Delta / (2 sigma_M)),
// lambda~ = lam_scale x the smaller eigenvalue of the 3 x 3 window sum of
// grad I1 grad I1^T, Delta = |I1(x) - I2(x')| + |grad I1(x) - grad I2(x')|.
__global__ void k_df_phi(const float* __restrict__ I1, const float* __restrict__ I2, PhiArgs a,
                         const dm_match* __restrict__ m, const int* __restrict__ n_matches, float* __restrict__ phi) {
    const int i = blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= min(*n_matches, a.max_matches)) return;   // the count never reaches past the caller's arrays
    const int x1 = clampi(m[i].x1, 0, a.W - 1), y1 = clampi(m[i].y1, 0, a.H - 1);
    const int x2 = clampi(m[i].x2, 0, a.W - 1), y2 = clampi(m[i].y2, 0, a.H - 1);
    float s11 = 0.f, s12 = 0.f, s22 = 0.f;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            float gx, gy;
            grad_at(I1, a.W, a.H, clampi(x1 + dx, 0, a.W - 1), clampi(y1 + dy, 0, a.H - 1), gx, gy);
            gx *= 255.f;
            gy *= 255.f;
            s11 += gx * gx;
            s12 += gx * gy;
            s22 += gy * gy;
        }
    const float lam = 0.5f * (s11 + s22) - sqrtf(0.25f * (s11 - s22) * (s11 - s22) + s12 * s12);
    float g1x, g1y, g2x, g2y;
    grad_at(I1, a.W, a.H, x1, y1, g1x, g1y);
    grad_at(I2, a.W, a.H, x2, y2, g2x, g2y);
    const float delta = 255.f * (fabsf(I1[(size_t)y1 * a.W + x1] - I2[(size_t)y2 * a.W + x2]) +
                                 sqrtf((g1x - g2x) * (g1x - g2x) + (g1y - g2y) * (g1y - g2y)));
    phi[i] = sqrtf(a.lam_scale * fmaxf(lam, 0.f)) / (a.sigma_m * 2.5066282746310002f) * expf(-delta / (2.f * a.sigma_m));
}

struct FieldArgs {
    int W, H, Wk, Hk, max_matches;
    float sx, sy;
};

// Level pixel of a match's source: the nearest to (x1 + 0.5) Wk / W - 0.5,
// i.e. floor((2 x1 + 1) Wk / (2 W)), in exact integer arithmetic.
__device__ inline int level_pixel(const dm_match& q, const FieldArgs& a) {
    const int xk = clampi((int)(((2ll * q.x1 + 1) * a.Wk) / (2ll * a.W)), 0, a.Wk - 1);
    const int yk = clampi((int)(((2ll * q.y1 + 1) * a.Hk) / (2ll * a.H)), 0, a.Hk - 1);
    return yk * a.Wk + xk;
}

// The first match (smallest index) landing on each level pixel owns it
// (owner holds 0x7fffffff everywhere before: filled once per call, and
// reset by k_df_field where it reads).
__global__ void k_df_owner(const dm_match* __restrict__ m, const int* __restrict__ n_matches, FieldArgs a,
                           int* __restrict__ owner) {
    const int i = blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= min(*n_matches, a.max_matches)) return;
    atomicMin(&owner[level_pixel(m[i], a)], i);
}
__global__ void k_df_field(const dm_match* __restrict__ m, const float* __restrict__ phi,
                           int* __restrict__ owner, FieldArgs a, float* __restrict__ up, float* __restrict__ vp,
                           float* __restrict__ cphi) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= (long)a.Wk * a.Hk) return;
    const int o = owner[i];
    owner[i] = 0x7fffffff;   // clean for the next level's owners
    if (o == 0x7fffffff) {
        up[i] = vp[i] = cphi[i] = 0.f;
        return;
    }
    up[i] = (float)(m[o].x2 - m[o].x1) * a.sx;
    vp[i] = (float)(m[o].y2 - m[o].y1) * a.sy;
    cphi[i] = phi[o];
}

// ---------------------------------------------------------------- one level
struct LevelMaps {
    int W, H;
    const float *I1, *I2;
    float *u, *v, *du, *dv, *up, *vp, *cphi;
    float *I2w, *Ax, *Ay, *It, *Ixt, *Iyt, *alpha;
    float* J;    // 12 planes: J0 (11, 12, 13, 22, 23, 33), then Jxy
    float* A;    // 5 planes: a11 - G, a12, a22 - G, b1 + G u, b2 + G v (the frozen system without the edges)
    float* sw;   // alpha psi' of the smoothness term per pixel
};

// Per-pixel steps of a level (pixel i of L.W x L.H), shared by the
// one-launch-per-step kernels of large levels and the one-workgroup kernel of
// small ones.

// I2 warped by the current flow (bilinear, clamped).
__device__ inline void px_warp(const LevelMaps& L, long i) {
    const int y = (int)(i / L.W), x = (int)(i - (long)y * L.W);
    L.I2w[i] = bilinear(L.I2, L.W, L.H, (float)x + L.u[i], (float)y + L.v[i]);
}

// First derivatives: of A = (I1 + I2w) / 2 (spatial), I2w - I1 (temporal),
// the difference of the images' spatial derivatives (I_xt, I_yt), and
// alpha(x) = exp(-kappa |grad I1|).
__device__ inline void px_grad1(const LevelMaps& L, long i, float kappa) {
    const int W = L.W, H = L.H;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    const long l = (long)y * W + max(x - 1, 0), r = (long)y * W + min(x + 1, W - 1);
    const long t = (long)max(y - 1, 0) * W + x, b = (long)min(y + 1, H - 1) * W + x;
    const float g1x = 0.5f * (L.I1[r] - L.I1[l]), g1y = 0.5f * (L.I1[b] - L.I1[t]);
    const float g2x = 0.5f * (L.I2w[r] - L.I2w[l]), g2y = 0.5f * (L.I2w[b] - L.I2w[t]);
    const float Ar = 0.5f * (L.I1[r] + L.I2w[r]), Al = 0.5f * (L.I1[l] + L.I2w[l]);
    const float Ab = 0.5f * (L.I1[b] + L.I2w[b]), At = 0.5f * (L.I1[t] + L.I2w[t]);
    L.Ax[i] = 0.5f * (Ar - Al);
    L.Ay[i] = 0.5f * (Ab - At);
    L.It[i] = L.I2w[i] - L.I1[i];
    L.Ixt[i] = g2x - g1x;
    L.Iyt[i] = g2y - g1y;
    L.alpha[i] = expf(-kappa * sqrtf(g1x * g1x + g1y * g1y));
}

// Normalised data tensors (Eq. (18)): J0 from (A_x, A_y, I_t), Jxy from
// (A_xx, A_xy, I_xt) and (A_xy, A_yy, I_yt), second derivatives being central
// differences of the first (replicated borders).
__device__ inline void px_tensors(const LevelMaps& L, long i, float zeta) {
    const long n = (long)L.W * L.H;
    const int W = L.W, H = L.H;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    const long l = (long)y * W + max(x - 1, 0), r = (long)y * W + min(x + 1, W - 1);
    const long t = (long)max(y - 1, 0) * W + x, b = (long)min(y + 1, H - 1) * W + x;
    const float ax = L.Ax[i], ay = L.Ay[i], it = L.It[i];
    const float axx = 0.5f * (L.Ax[r] - L.Ax[l]), axy = 0.5f * (L.Ax[b] - L.Ax[t]);
    const float ayy = 0.5f * (L.Ay[b] - L.Ay[t]);
    const float ixt = L.Ixt[i], iyt = L.Iyt[i];
    const float z2 = zeta * zeta;
    const float t0 = 1.f / (ax * ax + ay * ay + z2);
    const float tx = 1.f / (axx * axx + axy * axy + z2), ty = 1.f / (axy * axy + ayy * ayy + z2);
    float* J = L.J;
    J[0 * n + i] = t0 * ax * ax;
    J[1 * n + i] = t0 * ax * ay;
    J[2 * n + i] = t0 * ax * it;
    J[3 * n + i] = t0 * ay * ay;
    J[4 * n + i] = t0 * ay * it;
    J[5 * n + i] = t0 * it * it;
    J[6 * n + i] = tx * axx * axx + ty * axy * axy;
    J[7 * n + i] = tx * axx * axy + ty * axy * ayy;
    J[8 * n + i] = tx * axx * ixt + ty * axy * iyt;
    J[9 * n + i] = tx * axy * axy + ty * ayy * ayy;
    J[10 * n + i] = tx * axy * ixt + ty * ayy * iyt;
    J[11 * n + i] = tx * ixt * ixt + ty * iyt * iyt;
}

struct WeightArgs {
    float gamma, delta, eps, beta_k;
};

// One fixed-point step: the penalisers' derivatives at the current
// increment, and the frozen system without its edge terms.
__device__ inline void px_weights(const LevelMaps& L, long i, const WeightArgs& w) {
    const long n = (long)L.W * L.H;
    const int W = L.W, H = L.H;
    const int y = (int)(i / W), x = (int)(i - (long)y * W);
    const float du = L.du[i], dv = L.dv[i];
    const float* J = L.J;
    auto quad = [&](int o) {
        return J[(o + 0) * n + i] * du * du + 2.f * J[(o + 1) * n + i] * du * dv + 2.f * J[(o + 2) * n + i] * du +
               J[(o + 3) * n + i] * dv * dv + 2.f * J[(o + 4) * n + i] * dv + J[(o + 5) * n + i];
    };
    const float w0 = w.delta * psi_prime(quad(0), w.eps), wxy = w.gamma * psi_prime(quad(6), w.eps);
    float wJ[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) wJ[c] = w0 * J[c * n + i] + wxy * J[(6 + c) * n + i];
    const long l = (long)y * W + max(x - 1, 0), r = (long)y * W + min(x + 1, W - 1);
    const long t = (long)max(y - 1, 0) * W + x, b = (long)min(y + 1, H - 1) * W + x;
    auto U = [&](long k) { return L.u[k] + L.du[k]; };
    auto V = [&](long k) { return L.v[k] + L.dv[k]; };
    const float ux = 0.5f * (U(r) - U(l)), uy = 0.5f * (U(b) - U(t));
    const float vx = 0.5f * (V(r) - V(l)), vy = 0.5f * (V(b) - V(t));
    L.sw[i] = L.alpha[i] * psi_prime(ux * ux + uy * uy + vx * vx + vy * vy, w.eps);
    const float u = L.u[i], v = L.v[i];
    const float eu = u + du - L.up[i], ev = v + dv - L.vp[i];
    const float wM = w.beta_k * L.cphi[i] * psi_prime(eu * eu + ev * ev, w.eps);
    float* A = L.A;
    A[0 * n + i] = wJ[0] + wM;
    A[1 * n + i] = wJ[1];
    A[2 * n + i] = wJ[3] + wM;
    A[3 * n + i] = -wJ[2] - wM * (u - L.up[i]);
    A[4 * n + i] = -wJ[4] - wM * (v - L.vp[i]);
}

#define DF_PIXEL_KERNEL(name, body, ...)                              \
    __global__ void name(LevelMaps L, __VA_ARGS__) {                   \
        const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;   \
        if (i < (long)L.W * L.H) body;                                 \
    }
__global__ void k_df_warp(LevelMaps L) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i < (long)L.W * L.H) px_warp(L, i);
}
DF_PIXEL_KERNEL(k_df_grad1, px_grad1(L, i, kappa), float kappa)
DF_PIXEL_KERNEL(k_df_tensors, (px_tensors(L, i, zeta), L.du[i] = 0.f, L.dv[i] = 0.f), float zeta)
DF_PIXEL_KERNEL(k_df_weights, px_weights(L, i, w), WeightArgs w)
#undef DF_PIXEL_KERNEL

// ---------------------------------------------------------------- SOR
// Red-black block SOR: in one half-sweep every pixel of one colour
// ((x + y) % 2) solves its 2 x 2 block, with the edges to its (up to 4)
// neighbours, against the neighbours' current flow u + du, v + dv, and
// relaxes its increment by omega.  Same-colour pixels are never neighbours,
// so the pixels of a half-sweep are independent.  The frozen system does not
// change during the sweeps, so a pixel keeps its edge weights (0 for an edge
// leaving the level), the inverse of its matrix and the constant part of its
// right-hand side in registers, and reads its neighbours' flow from LDS.
struct SorPx {
    float u, v, du, dv;    // flow and increment
    float g[4];            // edge weights: left, right, top, bottom
    float i11, i12, i22;   // inverse of [[a11, a12], [a12, a22]]
    float r1b, r2b;        // right-hand side without the neighbours' flow
};

// sc: the pixel's alpha psi'; sn[k]: its neighbours' (ignored where ex[k] is
// false); A: the pixel's five entries of the frozen system without edges.
__device__ inline void sor_px_init(SorPx& p, float sc, const float (&sn)[4], const bool (&ex)[4],
                                   const float (&A)[5]) {
    float G = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        p.g[k] = ex[k] ? 0.5f * (sc + sn[k]) : 0.f;
        G += p.g[k];
    }
    const float a11 = A[0] + G, a12 = A[1], a22 = A[2] + G;
    const float rdet = 1.f / (a11 * a22 - a12 * a12);   // > 0: G > 0 and the data part is semi-definite
    p.i11 = a22 * rdet;
    p.i12 = a12 * rdet;
    p.i22 = a11 * rdet;
    p.r1b = A[3] - G * p.u;
    p.r2b = A[4] - G * p.v;
}

// One update from the neighbours' flow nb (left, right, top, bottom; any
// finite value where the edge weight is 0); returns the new u + du, v + dv.
__device__ inline float2 sor_px_update(SorPx& p, const float2 (&nb)[4], float omega) {
    float su = 0.f, sv = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        su += p.g[k] * nb[k].x;
        sv += p.g[k] * nb[k].y;
    }
    const float r1 = p.r1b + su, r2 = p.r2b + sv;
    const float nu = p.i11 * r1 - p.i12 * r2, nv = p.i22 * r2 - p.i12 * r1;
    p.du += omega * (nu - p.du);
    p.dv += omega * (nv - p.dv);
    return make_float2(p.u + p.du, p.v + p.dv);
}

__device__ inline void load_system(const LevelMaps& L, long n, long i, float (&A)[5]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) A[c] = L.A[c * n + i];
}

// Tiled levels: several half-sweeps per launch.  A workgroup holds a tile of
// LX x LY pixels on chip, runs up to HALO half-sweeps on it and writes back
// the inner (LX - 2 HALO) x (LY - 2 HALO) pixels.  A pixel with a neighbour
// inside the level but outside the tile is never updated; the error this
// leaves moves one pixel inward per half-sweep, so after at most HALO
// half-sweeps every inner pixel holds what the same half-sweeps over the
// whole level give.  The increments go from one buffer to another, since a
// tile's rim overlaps other tiles' inner pixels.  Thread t owns the two
// columns 2 (t % 32) + {0, 1} of two consecutive rows: a 2 x 2 block, two
// pixels of each colour, so each half-sweep updates one pixel per row and
// thread, and two of an updated pixel's four neighbours (the other pixel of
// its row, the other row's pixel of its column) are the thread's own, read
// from registers.  Inner sizes are even, so the tile origin X0 + Y0 is even
// and a pixel's colour is that of its position in the tile, known at
// compile time.
//
// A launch costs about 6 us whatever it does (start, loads, stores) plus
// 0.3 to 0.5 us per half-sweep, so a level's 2 n_sor half-sweeps per fixed
// point want few launches: 1024 threads on 64 x 64 tiles with a rim of 25
// (two launches for 25 sweeps) or 17 (three) where the tiles fit the chip
// at once, else 512 threads on 64 x 32 tiles with a rim of 10 (five).
template <int THREADS, int HALO>
struct SorTile {
    static constexpr int RIM = HALO;                 // half-sweeps per launch at most
    static constexpr int CP = 32;                    // column pairs per tile row
    static constexpr int LX = 2 * CP;                // tile columns
    static constexpr int LY = THREADS / CP * 2;      // tile rows (two per thread)
    static constexpr int IX = LX - 2 * HALO;         // inner columns
    static constexpr int IY = LY - 2 * HALO;         // inner rows
    static_assert(IX > 0 && IY > 0 && IX % 2 == 0 && IY % 2 == 0, "inner sizes must be even");
};
using SorNarrow = SorTile<512, 10>;
using SorWide = SorTile<1024, 25>;
using SorMid = SorTile<1024, 17>;

struct SorArgs {
    int ntx;     // tiles along x
    int nhalf;   // half-sweeps of this launch, at most the tile's rim
    int c0;      // colour of the first half-sweep
    float omega;
    const float *du_in, *dv_in;
    float *du_out, *dv_out;
    float *u_fin, *v_fin;   // last launch of the level: the level's flow u + du, v + dv goes here instead
};

template <int THREADS, int HALO>
__global__ __launch_bounds__(THREADS) void k_df_sor_tiles(LevelMaps L, SorArgs a) {
    using T = SorTile<THREADS, HALO>;
    constexpr int LX = T::LX, LY = T::LY;
    __shared__ float2 sUV[LY + 2][LX + 2];   // u + du, v + dv; a zero border
    __shared__ float sS[LY + 2][LX + 2];     // alpha psi' (0 outside the level)
    const int W = L.W, H = L.H;
    const long n = (long)W * H;
    const int tx = blockIdx.x % a.ntx, ty = blockIdx.x / a.ntx;
    const int X0 = tx * T::IX - HALO, Y0 = ty * T::IY - HALO;
    const int t = threadIdx.x, cp = t % T::CP, rg = t / T::CP;
    for (int e = t; e < 2 * (LX + 2) + 2 * LY; e += THREADS) {
        int yy, xx;
        if (e < 2 * (LX + 2)) {
            yy = e < LX + 2 ? 0 : LY + 1;
            xx = e % (LX + 2);
        } else {
            const int k = e - 2 * (LX + 2);
            yy = 1 + (k >> 1);
            xx = (k & 1) ? LX + 1 : 0;
        }
        sUV[yy][xx] = make_float2(0.f, 0.f);
        sS[yy][xx] = 0.f;
    }
    SorPx q[2][2];
    float2 w[2][2];   // u + du, v + dv of the thread's pixels (what sUV holds for them)
    bool upd[2][2];
    float Av[2][2][5];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * cp + j, ly = 2 * rg + r, x = X0 + lx, y = Y0 + ly;
            const bool in = x >= 0 && x < W && y >= 0 && y < H;
            // updated: inside the level, every neighbour inside the level lies inside the tile
            upd[r][j] = in && (x == 0 || lx > 0) && (x + 1 == W || lx + 1 < LX) && (y == 0 || ly > 0) &&
                        (y + 1 == H || ly + 1 < LY);
            const long i = in ? (long)y * W + x : 0;
            SorPx& p = q[r][j];
            p.u = in ? L.u[i] : 0.f;
            p.v = in ? L.v[i] : 0.f;
            p.du = in ? a.du_in[i] : 0.f;
            p.dv = in ? a.dv_in[i] : 0.f;
            if (upd[r][j]) load_system(L, n, i, Av[r][j]);
            w[r][j] = make_float2(p.u + p.du, p.v + p.dv);
            sUV[ly + 1][lx + 1] = w[r][j];
            sS[ly + 1][lx + 1] = in ? L.sw[i] : 0.f;
        }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (!upd[r][j]) continue;
            const int lx = 2 * cp + j, ly = 2 * rg + r, x = X0 + lx, y = Y0 + ly;
            const float sn[4] = {sS[ly + 1][lx], sS[ly + 1][lx + 2], sS[ly][lx + 1], sS[ly + 2][lx + 1]};
            const bool ex[4] = {x > 0, x + 1 < W, y > 0, y + 1 < H};
            sor_px_init(q[r][j], sS[ly + 1][lx + 1], sn, ex, Av[r][j]);
        }
    // Distance (rows or columns, the larger) of each pixel from the inner
    // region: a value computed at a half-sweep after which R half-sweeps
    // remain reaches at most R pixels further, so a pixel farther than R from
    // the inner region is left as it is (whole waves skip the rows that are).
    auto dist = [&](int v, int inner) { return max(max(HALO - v, v - (HALO + inner - 1)), 0); };
    int far[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 2; ++j) far[r][j] = max(dist(2 * rg + r, T::IY), dist(2 * cp + j, T::IX));
    // One half-sweep of colour C (the hh-th of the launch): the pixel of
    // colour C in row r is column j = (C + r) & 1; the other pixel of its row
    // and the other row's pixel of its column are of the other colour and the
    // thread's own.
    auto half = [&](auto cc, int hh) {
        constexpr int C = decltype(cc)::value;
        const int R = a.nhalf - 1 - hh;
        if (min(far[0][C & 1], far[1][(C + 1) & 1]) <= R) {
            float2 nb[2][4];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = (C + r) & 1, lx = 2 * cp + j, ly = 2 * rg + r;
                const float2 side = j ? sUV[ly + 1][lx + 2] : sUV[ly + 1][lx];   // the neighbour outside the block
                const float2 vert = r ? sUV[ly + 2][lx + 1] : sUV[ly][lx + 1];
                nb[r][0] = j ? w[r][0] : side;       // left
                nb[r][1] = j ? side : w[r][1];       // right
                nb[r][2] = r ? w[0][j] : vert;       // top
                nb[r][3] = r ? vert : w[1][j];       // bottom
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int j = (C + r) & 1, lx = 2 * cp + j, ly = 2 * rg + r;
                if (upd[r][j] && far[r][j] <= R) {
                    w[r][j] = sor_px_update(q[r][j], nb[r], a.omega);
                    sUV[ly + 1][lx + 1] = w[r][j];
                }
            }
        }
        __syncthreads();
    };
    int h = 0;
    if (a.c0) {
        half(std::integral_constant<int, 1>(), 0);
        h = 1;
    }
    for (; h + 2 <= a.nhalf; h += 2) {
        half(std::integral_constant<int, 0>(), h);
        half(std::integral_constant<int, 1>(), h + 1);
    }
    if (h < a.nhalf) half(std::integral_constant<int, 0>(), h);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * cp + j, ly = 2 * rg + r, x = X0 + lx, y = Y0 + ly;
            if (lx < HALO || lx >= HALO + T::IX || ly < HALO || ly >= HALO + T::IY || x >= W || y >= H) continue;
            const long i = (long)y * W + x;
            if (a.u_fin) {
                a.u_fin[i] = q[r][j].u + q[r][j].du;
                a.v_fin[i] = q[r][j].v + q[r][j].dv;
            } else {
                a.du_out[i] = q[r][j].du;
                a.dv_out[i] = q[r][j].dv;
            }
        }
}

// A whole level in one workgroup (small and mid-size levels): every step of
// the level in order, each a block-stride loop over the pixels, a barrier
// between steps (the workgroup's global-memory writes are visible to it after
// a barrier).  The SOR of each fixed point runs on chip.  Thread t owns the
// pixel pairs (2 p, 2 p + 1), p = t + 1024 k: two consecutive pixels in
// raster order are always of different colours (in one row they are
// neighbours; across a row end of an odd width W, W - 1 is even), so slot c
// of a pair holds its pixel of colour c and every lane updates one pixel per
// pair and half-sweep.  A slot's whole state stays in registers; u + du,
// v + dv of the level sit in LDS split by colour, the pixel of colour c of
// pair p at uv[c][p], so a half-sweep writes uv[c] and reads only uv[1 - c].
// A pixel's horizontal neighbour inside its own pair is the thread's other
// slot, read from registers.
constexpr int kDfSmallThreads = 1024;
constexpr long kDfSmallPixels = 4096;                                        // levels up to this size run here
constexpr int kDfSmallPairs = (int)(kDfSmallPixels / 2 / kDfSmallThreads);   // pixel pairs per thread

struct SmallLDS {
    float2 uv[2][kDfSmallPixels / 2];   // u + du, v + dv by colour and pair
    float s[kDfSmallPixels];            // alpha psi' by pixel
};

__device__ inline void sor_level_small(const LevelMaps& L, int n_sor, float omega, SmallLDS& S) {
    const int W = L.W, H = L.H, n = W * H, np = (n + 1) / 2;
    // An opaque copy of the thread index: the pixel indices and addresses
    // derived from it are recomputed at each call rather than kept live
    // across the caller's other steps (which would spill registers).
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    SorPx q[kDfSmallPairs][2];
    int px[kDfSmallPairs][2];   // pixel of the slot, -1: none
    int nx[kDfSmallPairs][2];   // pair of the horizontal neighbour outside the pair
    int nu[kDfSmallPairs][2];   // pairs of the top and bottom neighbours (the own pair where none)
    int nd[kDfSmallPairs][2];
    bool sd[kDfSmallPairs][2];  // the slot is the second pixel of its pair
#pragma unroll
    for (int k = 0; k < kDfSmallPairs; ++k) {
        const int p = t + k * kDfSmallThreads, i0 = 2 * p;
        const int y0 = i0 / W, c0 = (i0 - y0 * W + y0) & 1;   // colour of pixel i0
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = i0 + (c0 ^ c);
            px[k][c] = i < n ? i : -1;
            if (p >= np) continue;
            SorPx& r = q[k][c];
            r.u = r.v = r.du = r.dv = 0.f;   // the missing second pixel of an odd-sized level: a finite 0
            if (i < n) {
                r.u = L.u[i];
                r.v = L.v[i];
                r.du = L.du[i];
                r.dv = L.dv[i];
                S.s[i] = L.sw[i];
            }
            S.uv[c][p] = make_float2(r.u + r.du, r.v + r.dv);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kDfSmallPairs; ++k)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = px[k][c], p = t + k * kDfSmallThreads;
            if (i < 0) continue;
            const int y = i / W, x = i - y * W;
            const bool e[4] = {x > 0, x + 1 < W, y > 0, y + 1 < H};
            const float sn[4] = {S.s[e[0] ? i - 1 : i], S.s[e[1] ? i + 1 : i], S.s[e[2] ? i - W : i],
                                 S.s[e[3] ? i + W : i]};
            float A[5];
            load_system(L, n, i, A);
            sor_px_init(q[k][c], S.s[i], sn, e, A);
            // a neighbour that does not exist has edge weight 0: any finite value serves,
            // the own pair's entry of the other colour is one
            sd[k][c] = i & 1;
            nx[k][c] = (i & 1) ? (e[1] ? p + 1 : p) : (e[0] ? p - 1 : p);
            nu[k][c] = e[2] ? (i - W) >> 1 : p;
            nd[k][c] = e[3] ? (i + W) >> 1 : p;
        }
    for (int it = 0; it < n_sor; ++it)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // a pixel's neighbours are of the other colour: no update of this
            // half-sweep changes them
            const float2* o = S.uv[1 - c];
#pragma unroll
            for (int k = 0; k < kDfSmallPairs; ++k) {
                if (px[k][c] < 0) continue;
                const SorPx& m = q[k][1 - c];
                const float2 own = make_float2(m.u + m.du, m.v + m.dv);   // the pair's other pixel
                const float2 h = o[nx[k][c]];
                const float2 nb[4] = {sd[k][c] ? own : h, sd[k][c] ? h : own, o[nu[k][c]], o[nd[k][c]]};
                S.uv[c][t + k * kDfSmallThreads] = sor_px_update(q[k][c], nb, omega);
            }
            __syncthreads();
        }
#pragma unroll
    for (int k = 0; k < kDfSmallPairs; ++k)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int i = px[k][c];
            if (i < 0) continue;
            L.du[i] = q[k][c].du;
            L.dv[i] = q[k][c].dv;
        }
    __syncthreads();
}

__global__ __launch_bounds__(kDfSmallThreads) void k_df_level_small(LevelMaps L, float kappa, float zeta,
                                                                     WeightArgs w, int n_fixed, int n_sor,
                                                                     float omega) {
    __shared__ SmallLDS S;
    const long n = (long)L.W * L.H;
    const long t = threadIdx.x;
#define DF_ALL(stmt)                                               \
    do {                                                           \
        for (long i = t; i < n; i += kDfSmallThreads) { stmt; }    \
        __syncthreads();                                           \
    } while (0)
    DF_ALL(px_warp(L, i));
    DF_ALL(px_grad1(L, i, kappa));
    DF_ALL((px_tensors(L, i, zeta), L.du[i] = 0.f, L.dv[i] = 0.f));
    for (int f = 0; f < n_fixed; ++f) {
        DF_ALL(px_weights(L, i, w));
        sor_level_small(L, n_sor, omega, S);
    }
    DF_ALL((L.u[i] += L.du[i], L.v[i] += L.dv[i]));
#undef DF_ALL
}

__global__ void k_df_add(float* __restrict__ u, float* __restrict__ v, const float* __restrict__ du,
                         const float* __restrict__ dv, long n) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= n) return;
    u[i] += du[i];
    v[i] += dv[i];
}

// Flow (H x W x 2, interleaved) from the finest level's u, v.
__global__ void k_df_pack(const float* __restrict__ u, const float* __restrict__ v, long n, float* __restrict__ flow) {
    const long i = (long)blockIdx.x * kDfThreads + threadIdx.x;
    if (i >= n) return;
    flow[2 * i] = u[i];
    flow[2 * i + 1] = v[i];
}

// ---------------------------------------------------------------- plan
struct FlowLayout {
    std::vector<int> W, H;     // level sizes, 0 = finest
    std::vector<size_t> off1, off2;   // pyramid images of each level
    size_t u, v, u2, v2, du, dv, du2, dv2, up, vp, cphi, owner, I2w, Ax, Ay, It, Ixt, Iyt, alpha, J, A, sw, phi, tmp;
    size_t total;
};

inline size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

bool flow_levels(int W, int H, const dm_flow_params& p, std::vector<int>& Ws, std::vector<int>& Hs) {
    Ws.assign(1, W);
    Hs.assign(1, H);
    for (int k = 1;; ++k) {
        const int w = (int)floor(W * pow((double)p.eta, (double)k) + 0.5);
        const int h = (int)floor(H * pow((double)p.eta, (double)k) + 0.5);
        if (w < p.min_size || h < p.min_size) break;
        if ((int)Ws.size() >= DM_FLOW_MAX_LEVELS) return false;
        Ws.push_back(w);
        Hs.push_back(h);
    }
    return true;
}

dm_status flow_layout(int W, int H, int max_matches, const dm_flow_params& p, FlowLayout& L) {
    if (!flow_levels(W, H, p, L.W, L.H))
        return fail(DM_ERR_SHAPE, "more than %d pyramid levels (eta %g, min_size %d)", DM_FLOW_MAX_LEVELS,
                    (double)p.eta, p.min_size);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = a256(o + bytes);
        return r;
    };
    const size_t n = (size_t)W * H;
    for (size_t k = 0; k < L.W.size(); ++k) {
        L.off1.push_back(take((size_t)L.W[k] * L.H[k] * 4));
        L.off2.push_back(take((size_t)L.W[k] * L.H[k] * 4));
    }
    L.u = take(n * 4), L.v = take(n * 4), L.u2 = take(n * 4), L.v2 = take(n * 4);
    L.du = take(n * 4), L.dv = take(n * 4), L.du2 = take(n * 4), L.dv2 = take(n * 4);
    L.up = take(n * 4), L.vp = take(n * 4), L.cphi = take(n * 4);
    L.owner = take(n * 4), L.I2w = take(n * 4), L.Ax = take(n * 4), L.Ay = take(n * 4), L.It = take(n * 4);
    L.Ixt = take(n * 4), L.Iyt = take(n * 4), L.alpha = take(n * 4), L.J = take(12 * n * 4), L.A = take(5 * n * 4);
    L.sw = take(n * 4), L.phi = take((size_t)(max_matches > 0 ? max_matches : 1) * 4), L.tmp = take(n * 4);
    L.total = o + 256;
    return DM_OK;
}

dm_status check_flow_params(const dm_flow_params* p) {
    if (!p) return fail(DM_ERR_INVALID_ARG, "flow params pointer is null");
    if (!(p->sigma > 0.f) || (int)ceilf(3.f * p->sigma) > kDfMaxRadius)
        return fail(DM_ERR_INVALID_ARG, "sigma must lie in (0, %g]", kDfMaxRadius / 3.0);
    if (!(p->eta > 0.f && p->eta < 1.f)) return fail(DM_ERR_INVALID_ARG, "eta must lie in (0, 1)");
    if (p->min_size < 2) return fail(DM_ERR_INVALID_ARG, "min_size must be at least 2");
    if (p->n_fixed < 0 || p->n_sor < 0 || p->n_fixed > 1000 || p->n_sor > 10000)
        return fail(DM_ERR_INVALID_ARG, "iteration counts out of range");
    if (!(p->omega > 0.f && p->omega < 2.f)) return fail(DM_ERR_INVALID_ARG, "omega must lie in (0, 2)");
    if (!(p->eps > 0.f) || !(p->zeta > 0.f) || !(p->sigma_m > 0.f) || p->kappa < 0.f || p->beta < 0.f ||
        p->gamma < 0.f || p->delta < 0.f || p->lam_scale < 0.f)
        return fail(DM_ERR_INVALID_ARG, "negative weight or non-positive eps, zeta or sigma_M");
    return DM_OK;
}

}  // namespace
}  // namespace dm

using namespace dm;

extern "C" {

dm_status dm_flow_default_params(dm_flow_params* p) {
    clear_error();
    if (!p) return fail(DM_ERR_INVALID_ARG, "params pointer is null");
    memset(p, 0, sizeof(*p));
    p->sigma = 0.5f;
    p->eta = 0.95f;
    p->min_size = 16;
    p->n_fixed = 5;
    p->n_sor = 25;
    p->omega = 1.6f;
    p->kappa = 5.f;
    p->beta = 300.f;
    p->b = 0.6f;
    p->gamma = 0.8f;
    p->delta = 0.f;
    p->eps = 0.001f;
    p->zeta = 0.1f;
    p->sigma_m = 50.f;
    p->lam_scale = 10.f;
    return DM_OK;
}

dm_status dm_flow_plan(int W, int H, int max_matches, const dm_flow_params* p, dm_flow_info* out) {
    clear_error();
    if (!out) return fail(DM_ERR_INVALID_ARG, "info pointer is null");
    dm_status st = check_flow_params(p);
    if (st != DM_OK) return st;
    if (W < 1 || H < 1 || (long long)W * H > (1ll << 26)) return fail(DM_ERR_SHAPE, "image size %d x %d", W, H);
    if (max_matches < 0) return fail(DM_ERR_INVALID_ARG, "max_matches is negative");
    FlowLayout L;
    if ((st = flow_layout(W, H, max_matches, *p, L)) != DM_OK) return st;
    memset(out, 0, sizeof(*out));
    out->n_levels = (int32_t)L.W.size();
    for (size_t k = 0; k < L.W.size(); ++k) {
        out->W[k] = L.W[k];
        out->H[k] = L.H[k];
    }
    out->workspace_bytes = L.total;
    return DM_OK;
}

}  // extern "C"

namespace dm {
namespace {

// The whole launch sequence of one DeepFlow call on stream s.
dm_status flow_enqueue(const float* img1, const float* img2, int W, int H, int ld, const dm_match* matches,
                       const int32_t* n_matches, int max_matches, const dm_flow_params* p, float* flow, void* ws,
                       hipStream_t s) {
    dm_status st = DM_OK;
    FlowLayout Lo;
    flow_layout(W, H, max_matches, *p, Lo);
    char* base = static_cast<char*>(ws);
    auto F = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
    const int K = (int)Lo.W.size() - 1;
    int dev = 0, n_cu = 0;
    if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice")) != DM_OK) return st;
    if ((st = check_hip(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev),
                        "hipDeviceGetAttribute")) != DM_OK)
        return st;
    Taps taps;
    {
        const int r = (int)ceil(3.0 * p->sigma);
        double k[2 * kDfMaxRadius + 1], sum = 0.0;
        for (int j = -r; j <= r; ++j) sum += (k[j + r] = exp(-(double)j * j / (2.0 * p->sigma * p->sigma)));
        for (int j = 0; j <= 2 * r; ++j) taps.k[j] = (float)(k[j] / sum);
        taps.r = r;
    }
#define DF(name, lvl, grid, ...)                                                    \
    do {                                                                            \
        timing_begin(name, lvl, s);                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                                            \
        timing_end(s);                                                              \
        if ((st = check_hip(hipGetLastError(), name)) != DM_OK) return st;          \
    } while (0)
    const long n0 = (long)W * H;
    // level 0 of the pyramid: the smoothed images
    DF("df_smooth", 0, 0, k_df_smooth_h, dim3(nblk(n0)), dim3(kDfThreads), 0, s, img1, W, H, ld, taps, F(Lo.tmp));
    DF("df_smooth", 0, 0, k_df_smooth_v, dim3(nblk(n0)), dim3(kDfThreads), 0, s, F(Lo.tmp), W, H, taps, F(Lo.off1[0]));
    DF("df_smooth", 0, 0, k_df_smooth_h, dim3(nblk(n0)), dim3(kDfThreads), 0, s, img2, W, H, ld, taps, F(Lo.tmp));
    DF("df_smooth", 0, 0, k_df_smooth_v, dim3(nblk(n0)), dim3(kDfThreads), 0, s, F(Lo.tmp), W, H, taps, F(Lo.off2[0]));
    if (max_matches > 0)
        DF("df_phi", -1, 0, k_df_phi, dim3(nblk(max_matches)), dim3(kDfThreads), 0, s, F(Lo.off1[0]), F(Lo.off2[0]),
           PhiArgs{W, H, max_matches, p->lam_scale, p->sigma_m}, matches, n_matches, F(Lo.phi));
    for (int k = 1; k <= K; ++k) {
        const long nk = (long)Lo.W[k] * Lo.H[k];
        const Resize2 r{{F(Lo.off1[k - 1]), F(Lo.off2[k - 1])}, {F(Lo.off1[k]), F(Lo.off2[k])}, {1.f, 1.f}};
        DF("df_pyramid", k, 0, k_df_resize2, dim3(nblk(nk)), dim3(kDfThreads), 0, s, r, Lo.W[k - 1], Lo.H[k - 1],
           Lo.W[k], Lo.H[k]);
    }
    DF("df_matches", -1, 0, k_df_fill_i32, dim3(nblk(n0)), dim3(kDfThreads), 0, s,
       reinterpret_cast<int*>(base + Lo.owner), n0, 0x7fffffff);
    float *u = F(Lo.u), *v = F(Lo.v), *u2 = F(Lo.u2), *v2 = F(Lo.v2);
    for (int k = K; k >= 0; --k) {
        const int Wk = Lo.W[k], Hk = Lo.H[k];
        const long nk = (long)Wk * Hk;
        const dim3 g(nblk(nk)), b(kDfThreads);
        if (k == K) {
            DF("df_init", k, 0, k_df_fill2, g, b, 0, s, u, v, nk, 0.f);
        } else {   // the flow of level k + 1 (u2, v2), resampled and scaled
            const Resize2 r{{u2, v2}, {u, v}, {(float)Wk / (float)Lo.W[k + 1], (float)Hk / (float)Lo.H[k + 1]}};
            DF("df_upsample", k, 0, k_df_resize2, g, b, 0, s, r, Lo.W[k + 1], Lo.H[k + 1], Wk, Hk);
        }
        const FieldArgs fa{W, H, Wk, Hk, max_matches, (float)Wk / (float)W, (float)Hk / (float)H};
        if (max_matches > 0)
            DF("df_matches", k, 0, k_df_owner, dim3(nblk(max_matches)), b, 0, s, matches, n_matches, fa,
               reinterpret_cast<int*>(base + Lo.owner));
        DF("df_matches", k, 0, k_df_field, g, b, 0, s, matches, F(Lo.phi), reinterpret_cast<int*>(base + Lo.owner),
           fa, F(Lo.up), F(Lo.vp), F(Lo.cphi));
        LevelMaps M{Wk,        Hk,        F(Lo.off1[k]), F(Lo.off2[k]), u,         v,           F(Lo.du),
                    F(Lo.dv),  F(Lo.up),  F(Lo.vp),      F(Lo.cphi),    F(Lo.I2w), F(Lo.Ax),    F(Lo.Ay),
                    F(Lo.It),  F(Lo.Ixt), F(Lo.Iyt),     F(Lo.alpha),   F(Lo.J),   F(Lo.A),     F(Lo.sw)};
        const float beta_k = (float)(p->beta * (K > 0 ? pow((double)k / K, (double)p->b) : 1.0));
        const WeightArgs wa{p->gamma, p->delta, p->eps, beta_k};
        if (nk <= kDfSmallPixels) {
            DF("df_level_small", k, 0, k_df_level_small, dim3(1), dim3(kDfSmallThreads), 0, s, M, p->kappa, p->zeta,
               wa, p->n_fixed, p->n_sor, p->omega);
        } else {
            DF("df_warp", k, 0, k_df_warp, g, b, 0, s, M);
            DF("df_grad", k, 0, k_df_grad1, g, b, 0, s, M, p->kappa);
            DF("df_tensors", k, 0, k_df_tensors, g, b, 0, s, M, p->zeta);   // also zeroes du, dv
            float *du_o = F(Lo.du2), *dv_o = F(Lo.dv2);   // the other increment buffers
            // the 64 x 64 shape with the fewest launches whose tiles fit the
            // compute units at once (on equal launches the larger inner region),
            // else the 64 x 32 one
            const int nh_fp = 2 * p->n_sor;
            auto launches = [&](int rim) { return (nh_fp + rim - 1) / rim; };
            auto tiles = [&](int ix, int iy) { return ((Wk + ix - 1) / ix) * ((Hk + iy - 1) / iy); };
            int shape = 0;   // 0: 64 x 32, rim 10; 1: 64 x 64, rim 17; 2: 64 x 64, rim 25
            if (tiles(SorMid::IX, SorMid::IY) <= n_cu) shape = 1;
            if (tiles(SorWide::IX, SorWide::IY) <= n_cu &&
                (shape == 0 || launches(SorWide::RIM) < launches(SorMid::RIM)))
                shape = 2;
            const int halo = shape == 2 ? SorWide::RIM : shape == 1 ? SorMid::RIM : SorNarrow::RIM;
            const int ix = shape == 2 ? SorWide::IX : shape == 1 ? SorMid::IX : SorNarrow::IX;
            const int iy = shape == 2 ? SorWide::IY : shape == 1 ? SorMid::IY : SorNarrow::IY;
            const int ntx = (Wk + ix - 1) / ix, nty = (Hk + iy - 1) / iy;
            bool flow_in_u2 = false;
            for (int f = 0; f < p->n_fixed; ++f) {
                DF("df_weights", k, 0, k_df_weights, g, b, 0, s, M, wa);
                for (int h = 0; h < 2 * p->n_sor; h += halo) {
                    const int nh = min(halo, 2 * p->n_sor - h);
                    // the level's last launch writes u + du, v + dv into u2, v2 (the coarser
                    // level's flow there has been resampled already)
                    const bool last = f + 1 == p->n_fixed && h + nh == 2 * p->n_sor;
                    const SorArgs sa{ntx, nh, h & 1, p->omega, M.du, M.dv, du_o, dv_o, last ? u2 : nullptr,
                                     last ? v2 : nullptr};
                    if (shape == 2)
                        DF("df_sor", k, 0, (k_df_sor_tiles<1024, SorWide::RIM>), dim3(ntx * nty), dim3(1024), 0, s, M,
                           sa);
                    else if (shape == 1)
                        DF("df_sor", k, 0, (k_df_sor_tiles<1024, SorMid::RIM>), dim3(ntx * nty), dim3(1024), 0, s, M,
                           sa);
                    else
                        DF("df_sor", k, 0, (k_df_sor_tiles<512, SorNarrow::RIM>), dim3(ntx * nty), dim3(512), 0, s, M,
                           sa);
                    std::swap(M.du, du_o);
                    std::swap(M.dv, dv_o);
                    flow_in_u2 = last;
                }
            }
            if (flow_in_u2) continue;   // u2, v2 hold level k's flow
            DF("df_add", k, 0, k_df_add, g, b, 0, s, u, v, M.du, M.dv, nk);   // no SOR sweeps: u + du
        }
        std::swap(u, u2);   // u2, v2 now hold level k's flow
        std::swap(v, v2);
    }
    DF("df_pack", 0, 0, k_df_pack, dim3(nblk(n0)), dim3(kDfThreads), 0, s, u2, v2, n0, flow);
#undef DF
    return DM_OK;
}

// Graphs of DM_FLOW_GRAPH calls, one per workspace, kept while the
// arguments stay the same.
struct FlowGraph {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~FlowGraph() {
        if (exec) {
            (void)hipDeviceSynchronize();   // a replay may still be running
            (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
};
std::mutex g_flow_mu;
std::map<const void*, std::unique_ptr<FlowGraph>> g_flow_graphs;

}  // namespace
}  // namespace dm

extern "C" {

dm_status dm_deepflow(const float* img1, const float* img2, int W, int H, int ld, const dm_match* matches,
                      const int32_t* n_matches, int max_matches, const dm_flow_params* p, int flags, float* flow,
                      void* ws, size_t ws_bytes, hipStream_t s) {
    clear_error();
    dm_flow_info info;
    dm_status st = dm_flow_plan(W, H, max_matches, p, &info);
    if (st != DM_OK) return st;
    if (!img1 || !img2 || !flow) return fail(DM_ERR_INVALID_ARG, "image or flow pointer is null");
    if (ld < W) return fail(DM_ERR_SHAPE, "leading dimension %d below the width %d", ld, W);
    if (max_matches > 0 && (!matches || !n_matches)) return fail(DM_ERR_INVALID_ARG, "match pointers are null");
    if (!ws) return fail(DM_ERR_INVALID_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < info.workspace_bytes)
        return fail(DM_ERR_WORKSPACE, "workspace holds %zu bytes, DeepFlow needs %llu", ws_bytes,
                    (unsigned long long)info.workspace_bytes);
    if (flags & ~DM_FLOW_GRAPH) return fail(DM_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (!(flags & DM_FLOW_GRAPH)) return flow_enqueue(img1, img2, W, H, ld, matches, n_matches, max_matches, p, flow, ws, s);
    if (!s) return fail(DM_ERR_INVALID_ARG, "DM_FLOW_GRAPH needs a stream other than the null stream");
    std::vector<unsigned char> key;
    auto put = [&](const void* q, size_t b) {
        const size_t o = key.size();
        key.resize(o + b);
        memcpy(key.data() + o, q, b);
    };
    const void* ptrs[6] = {img1, img2, matches, n_matches, flow, ws};
    const int dims[4] = {W, H, ld, max_matches};
    put(ptrs, sizeof ptrs);
    put(dims, sizeof dims);
    put(p, sizeof(*p));
    put(&ws_bytes, sizeof ws_bytes);
    std::lock_guard<std::mutex> lk(g_flow_mu);
    auto it = g_flow_graphs.find(ws);
    if (it == g_flow_graphs.end() || it->second->key != key) {
        std::unique_ptr<FlowGraph> fg(new FlowGraph());
        fg->key = key;
        if ((st = check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture")) != DM_OK)
            return st;
        timing_suppress(true);   // no timing events inside the graph
        const dm_status rs = flow_enqueue(img1, img2, W, H, ld, matches, n_matches, max_matches, p, flow, ws, s);
        timing_suppress(false);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (rs != DM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rs;
        }
        if ((st = check_hip(ec, "graph capture")) != DM_OK) return st;
        fg->graph = graph;
        if ((st = check_hip(hipGraphInstantiate(&fg->exec, graph, nullptr, nullptr, 0), "graph instantiate")) != DM_OK)
            return st;
        g_flow_graphs[ws] = std::move(fg);
        it = g_flow_graphs.find(ws);
    }
    return check_hip(hipGraphLaunch(it->second->exec, s), "graph launch");
}

dm_status dm_flow_release(const void* ws) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_flow_mu);
    g_flow_graphs.erase(ws);
    return DM_OK;
}

}  // extern "C"
