// Gradient of a loss on the top-level maps with respect to both descriptor
// fields: the adjoint of rectification (Eq. (11)), of the shifted average
// over existing children (Eqs. (10), (12)), of the max-pool/subsample
// (Eqs. (8)-(9), routed to the stored argmax) and of the bottom correlation
// (Eq. (3)).  The paper has no backward pass; this one is written by hand.
//
// Notation (pooled grids, as in the forward):
//   g'_l(P, r) = dL/dC'_l(P, r) * lambda * C'_l(P, r)^((lambda-1)/lambda)
// is the gradient with respect to the pre-rectification value A_l at the
// argmax position 2r + m_l(P, r) carried by the pooled entry r (all entries
// routed to one position share its value, so their contributions add).  Then
//   G_l(P, q)       = sum_{r: 2r + m_l(P, r) = q} g'_l(P, r)      (top: dC_top * R')
//   dC'_{l-1}(c, r) = sum_{i: P = c - 2^l o_i exists, r - o_i in map} G_l(P, r - o_i) / |V(P)|
//   g'_{l-1}(c, r)  = dC'_{l-1}(c, r) * lambda * C'_{l-1}(c, r)^((lambda-1)/lambda)
// and at the bottom dA_0(p, x) = sum_{r: 2r + m_0(p, r) = x} g'_0(p, r).
// Every sum runs in a fixed order: results are deterministic.
#include "dm_internal.h"

namespace dm {
namespace {

template <typename T>
__device__ inline T rect_grad_factor(T c, T lam) {
    // d(max(A,0)^lam)/dA written from the stored value c = A^lam.
    return c > T(0) ? lam * rect_pow(c, (lam - T(1)) / lam) : T(0);
}

struct BwdArgs {
    int l;
    int gxp, gyp, gxc, gyc;
    int h, w;      // maps of level l (= child pooled grid)
    int hu, wu;    // pooled grid of level l
    int is_top;
};

template <typename T>
__device__ inline T parent_grad(const BwdArgs& a, int pb, int pa, int qy, int qx, const T* __restrict__ dtop,
                                const T* __restrict__ top, const T* __restrict__ gp_cur,
                                const uint8_t* __restrict__ code_cur, T lam) {
    if (a.is_top) {
        const size_t o = (((size_t)pb * a.gxp + pa) * a.h + qy) * a.w + qx;
        return dtop[o] * rect_grad_factor(top[o], lam);
    }
    T acc = 0;
    const int y0 = (qy - 1) >> 1, x0 = (qx - 1) >> 1;  // floor((q-1)/2)
    for (int ry = y0; ry <= (qy + 1) >> 1; ++ry) {
        if (ry < 0 || ry >= a.hu) continue;
        const int my = qy - 2 * ry;
        if (my < -1 || my > 1) continue;
        for (int rx = x0; rx <= (qx + 1) >> 1; ++rx) {
            if (rx < 0 || rx >= a.wu) continue;
            const int mx = qx - 2 * rx;
            if (mx < -1 || mx > 1) continue;
            const size_t o = (((size_t)pb * a.gxp + pa) * a.hu + ry) * a.wu + rx;
            if (code_cur[o] == 3 * (my + 1) + (mx + 1)) acc += gp_cur[o];
        }
    }
    return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd_level(BwdArgs a, const T* __restrict__ dtop, const T* __restrict__ top,
                                                   const T* __restrict__ gp_cur, const uint8_t* __restrict__ code_cur,
                                                   const T* __restrict__ cp_prev, const uint8_t* __restrict__ vt,
                                                   Geom g, T lam, T* __restrict__ gp_prev) {
    const size_t n = (size_t)a.gxc * a.gyc * a.h * a.w;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int rx = i % a.w, ry = (i / a.w) % a.h;
    const int c = i / ((size_t)a.w * a.h);
    const int cb = c / a.gxc, ca = c - cb * a.gxc;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    if (!(vxc[ca] && vyc[cb])) {
        gp_prev[i] = T(0);
        return;
    }
    T acc = 0;
    for (int side = 0; side < 4; ++side) {
        const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;   // o_i, i = side
        const int pb = parent_index(a.l, cb, sy), pa = parent_index(a.l, ca, sx);
        if (pb < 0 || pb >= a.gyp || pa < 0 || pa >= a.gxp || !vxp[pa] || !vyp[pb]) continue;
        const int qy = ry - sy, qx = rx - sx;
        if (qy < 0 || qy >= a.h || qx < 0 || qx >= a.w) continue;
        // |V(P)|: existing children of the parent along each axis.
        int nx = 0, ny = 0;
        for (int s = -1; s <= 1; s += 2) {
            const int ccx = child_index(a.l, pa, s), ccy = child_index(a.l, pb, s);
            nx += ccx >= 0 && ccx < a.gxc && vxc[ccx];
            ny += ccy >= 0 && ccy < a.gyc && vyc[ccy];
        }
        acc += parent_grad(a, pb, pa, qy, qx, dtop, top, gp_cur, code_cur, lam) / T(nx * ny);
    }
    gp_prev[i] = acc * rect_grad_factor(cp_prev[i], lam);
}

}  // namespace

template <typename T>
hipError_t launch_bwd_level(int l, const T* dtop, const T* top, const T* gp_cur, const uint8_t* code_cur,
                            const T* cp_prev, const uint8_t* vt, const Geom& g, T lam, T* gp_prev, hipStream_t s) {
    BwdArgs a;
    a.l = l;
    a.gxp = g.gx[l];
    a.gyp = g.gy[l];
    a.gxc = g.gx[l - 1];
    a.gyc = g.gy[l - 1];
    a.h = g.h[l];
    a.w = g.w[l];
    a.hu = g.h[l + 1];
    a.wu = g.w[l + 1];
    a.is_top = (l == g.lmax);
    const size_t n = (size_t)a.gxc * a.gyc * a.h * a.w;
    hipLaunchKernelGGL(k_bwd_level<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, dtop, top, gp_cur,
                       code_cur, cp_prev, vt, g, lam, gp_prev);
    return hipGetLastError();
}

template hipError_t launch_bwd_level<float>(int, const float*, const float*, const float*, const uint8_t*,
                                            const float*, const uint8_t*, const Geom&, float, float*, hipStream_t);
template hipError_t launch_bwd_level<double>(int, const double*, const double*, const double*, const uint8_t*,
                                             const double*, const uint8_t*, const Geom&, double, double*,
                                             hipStream_t);

}  // namespace dm
