// Upper levels of the pyramid (Sec. 3.2, Eqs. (10)-(12), Algorithm 1):
//   A_l(p, q) = 1/|V(p)| sum_{i in V(p)} C'_{l-1}(p + 2^l o_i, q + o_i)
//   C_l = max(A_l, 0)^lambda;  C'_l = (S o P)(C_l) + argmax codes, or C_top.
// V(p) = the existing children (boundary rule of Sec. 3.2); a child read
// outside its map counts 0.  One launch per level.
//
// A block owns PB parents x a tile of TRo x TCo pooled outputs.  It first
// stages max(A, 0) on the (2TRo+1) x (2TCo+1) positions the pooling windows
// touch (each A value feeds up to 4 windows), then pools from LDS.  Child maps
// are read straight from global memory, coalesced along x; a child is shared
// by up to 4 parents, which neighbouring blocks read at the same time.
#include "dm_internal.h"

namespace dm {
namespace {

struct LevelArgs {
    int l;
    int gx, gy, gxc, gyc;  // lattices of this level and of the children's
    int h, w, hp, wp;      // maps of this level (C_l) and pooled (C'_l)
    int TRo, TCo, PB;      // tile: pooled rows, pooled cols, parents per block
    int n_pblk, n_rt;      // block grid factors
};

template <typename T>
struct Parent {
    int valid;
    int cb[2], ca[2];      // child lattice indices per side (-1 if missing)
    T inv;                 // 1/|V|
};

template <typename T>
__device__ inline Parent<T> parent_info(const LevelArgs& a, int P, const uint8_t* vxp, const uint8_t* vyp,
                                        const uint8_t* vxc, const uint8_t* vyc) {
    Parent<T> r;
    const int pb = P / a.gx, pa = P - pb * a.gx;
    r.valid = (P < a.gx * a.gy) && vxp[pa] && vyp[pb];
    int nx = 0, ny = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int s = 2 * k - 1;
        const int ca = child_index(a.l, pa, s), cb = child_index(a.l, pb, s);
        r.ca[k] = (ca >= 0 && ca < a.gxc && vxc[ca]) ? ca : -1;
        r.cb[k] = (cb >= 0 && cb < a.gyc && vyc[cb]) ? cb : -1;
        nx += r.ca[k] >= 0;
        ny += r.cb[k] >= 0;
    }
    r.inv = (nx * ny) ? T(1) / T(nx * ny) : T(0);
    return r;
}

// A_l(P, q) for q inside the map.
template <typename T>
__device__ inline T aggregate(const LevelArgs& a, const Parent<T>& pi, const T* __restrict__ prev, int qy,
                              int qx) {
    T acc = 0;
#pragma unroll
    for (int ky = 0; ky < 2; ++ky) {
        const int cb = pi.cb[ky];
        const int y = qy + 2 * ky - 1;
        if (cb < 0 || y < 0 || y >= a.h) continue;
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
            const int ca = pi.ca[kx];
            const int x = qx + 2 * kx - 1;
            if (ca < 0 || x < 0 || x >= a.w) continue;
            acc += prev[(((size_t)cb * a.gxc + ca) * a.h + y) * a.w + x];
        }
    }
    return acc * pi.inv;
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_pool(LevelArgs a, const T* __restrict__ prev,
                                                    const uint8_t* __restrict__ vt, Geom g, T lam,
                                                    T* __restrict__ cp, uint8_t* __restrict__ code) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sA = (T*)smem_raw;
    const int bid = blockIdx.x;
    const int pblk = bid % a.n_pblk, rest = bid / a.n_pblk;
    const int R0 = (rest % a.n_rt) * a.TRo, C0 = (rest / a.n_rt) * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    const int RW = 2 * a.TCo + 1, RA = (2 * a.TRo + 1) * RW;
    // Phase 1: stage max(A, 0) on the pooling footprint (-1 outside the map).
    for (int e = threadIdx.x; e < a.PB * RA; e += 256) {
        const int k = e / RA, rem = e - k * RA;
        const int qy = 2 * R0 - 1 + rem / RW, qx = 2 * C0 - 1 + rem % RW;
        const Parent<T> pi = parent_info<T>(a, pblk * a.PB + k, vxp, vyp, vxc, vyc);
        T v = T(-1);
        if (pi.valid && qy >= 0 && qy < a.h && qx >= 0 && qx < a.w) {
            const T A = aggregate(a, pi, prev, qy, qx);
            v = A > 0 ? A : T(0);
        }
        sA[e] = v;
    }
    __syncthreads();
    // Phase 2: 3x3 / stride-2 max-pool, first maximum in code order, rectify.
    for (int e = threadIdx.x; e < a.PB * a.TRo * a.TCo; e += 256) {
        const int k = e / (a.TRo * a.TCo), rem = e - k * (a.TRo * a.TCo);
        const int orow = rem / a.TCo, ocol = rem - orow * a.TCo;
        const int P = pblk * a.PB + k, r = R0 + orow, c = C0 + ocol;
        if (P >= a.gx * a.gy || r >= a.hp || c >= a.wp) continue;
        const int pb = P / a.gx, pa = P - pb * a.gx;
        if (!(vxp[pa] && vyp[pb])) continue;
        const T* s = sA + k * RA;
        T best = T(-1);
        int bk = 0;
#pragma unroll
        for (int my = -1; my <= 1; ++my) {
            const int y = 2 * r + my;
            if (y < 0 || y >= a.h) continue;
#pragma unroll
            for (int mx = -1; mx <= 1; ++mx) {
                const int x = 2 * c + mx;
                if (x < 0 || x >= a.w) continue;
                const T v = s[(2 * orow + 1 + my) * RW + 2 * ocol + 1 + mx];
                if (v > best) {
                    best = v;
                    bk = 3 * (my + 1) + (mx + 1);
                }
            }
        }
        const size_t o = ((size_t)P * a.hp + r) * a.wp + c;
        cp[o] = rect_pow(best, lam);
        code[o] = (uint8_t)bk;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_top(LevelArgs a, const T* __restrict__ prev,
                                                   const uint8_t* __restrict__ vt, Geom g, T lam,
                                                   T* __restrict__ top) {
    const int bid = blockIdx.x;
    const int pblk = bid % a.n_pblk, rest = bid / a.n_pblk;
    const int R0 = (rest % a.n_rt) * a.TRo, C0 = (rest / a.n_rt) * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    for (int e = threadIdx.x; e < a.PB * a.TRo * a.TCo; e += 256) {
        const int k = e / (a.TRo * a.TCo), rem = e - k * (a.TRo * a.TCo);
        const int qy = R0 + rem / a.TCo, qx = C0 + rem % a.TCo;
        const int P = pblk * a.PB + k;
        if (qy >= a.h || qx >= a.w) continue;
        const Parent<T> pi = parent_info<T>(a, P, vxp, vyp, vxc, vyc);
        if (!pi.valid) continue;
        const T A = aggregate(a, pi, prev, qy, qx);
        top[((size_t)P * a.h + qy) * a.w + qx] = rect_pow(A > 0 ? A : T(0), lam);
    }
}

}  // namespace

template <typename T>
hipError_t launch_level(int l, const T* prev, const uint8_t* vt, const Geom& g, T lam, T* cp, uint8_t* code,
                        T* top, hipStream_t s) {
    LevelArgs a;
    a.l = l;
    a.gx = g.gx[l];
    a.gy = g.gy[l];
    a.gxc = g.gx[l - 1];
    a.gyc = g.gy[l - 1];
    a.h = g.h[l];
    a.w = g.w[l];
    a.hp = g.h[l + 1];
    a.wp = g.w[l + 1];
    const bool is_top = (l == g.lmax);
    const int th = is_top ? a.h : a.hp, tw = is_top ? a.w : a.wp;
    a.TCo = tw < 64 ? tw : 64;
    a.TRo = 256 / a.TCo;
    if (a.TRo > th) a.TRo = th;
    if (a.TRo < 1) a.TRo = 1;
    a.PB = 256 / (a.TRo * a.TCo);
    if (a.PB < 1) a.PB = 1;
    const int np = a.gx * a.gy;
    a.n_pblk = (np + a.PB - 1) / a.PB;
    a.n_rt = (th + a.TRo - 1) / a.TRo;
    const int n_ct = (tw + a.TCo - 1) / a.TCo;
    const dim3 grid(a.n_pblk * a.n_rt * n_ct);
    if (is_top) {
        hipLaunchKernelGGL(k_level_top<T>, grid, dim3(256), 0, s, a, prev, vt, g, lam, top);
    } else {
        const size_t smem = (size_t)a.PB * (2 * a.TRo + 1) * (2 * a.TCo + 1) * sizeof(T);
        hipLaunchKernelGGL(k_level_pool<T>, grid, dim3(256), smem, s, a, prev, vt, g, lam, cp, code);
    }
    return hipGetLastError();
}

template hipError_t launch_level<float>(int, const float*, const uint8_t*, const Geom&, float, float*, uint8_t*,
                                        float*, hipStream_t);
template hipError_t launch_level<double>(int, const double*, const uint8_t*, const Geom&, double, double*,
                                         uint8_t*, double*, hipStream_t);

}  // namespace dm
