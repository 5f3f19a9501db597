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
#include "dm_group.h"

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
    int TR, TC, CB;            // tile rows, cols, children per block
    int n_cblk, n_rt;
    FastDiv f_t, f_tc, f_nr, f_rwd;   // divisions by TR*TC, TC, RH*RWd, RWd
};

__device__ inline int xcd_block(int nblocks) {
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Block: CB children x a TR x TC tile of their pooled grid.  For each child
// and side i (parent P = c - 2^l o_i), the parent's data covering the tile is
// staged in LDS: at the top the gradient G_top on q = r - o_i, below the
// pooled gradient g'_l and codes on the r' whose argmax can land there.
template <typename T>
__device__ inline void bwd_level_body(const BwdArgs& a, const T* __restrict__ dtop, const T* __restrict__ top,
                                      const T* __restrict__ gp_cur, const uint8_t* __restrict__ code_cur,
                                      const T* __restrict__ cp_prev, const uint8_t* __restrict__ vt, const Geom& g,
                                      T lam, T* __restrict__ gp_prev, int bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int RH = a.TR / 2 + 2, RWd = a.TC / 2 + 2, NR = RH * RWd;
    const int T_ = a.TR * a.TC;
    const int per_side = a.is_top ? T_ : NR;
    T* sG = (T*)smem_raw;                                                  // [CB*4][per_side]
    uint8_t* sM = (uint8_t*)(sG + 4 * a.CB * per_side);                    // codes (below the top)
    int* sPar = (int*)(((uintptr_t)(sM + 4 * a.CB * per_side) + 15) & ~(uintptr_t)15);  // [CB*4]
    T* sInv = (T*)(sPar + 4 * a.CB);                                       // [CB*4] 1/|V(P)|
    int* sCv = (int*)(sInv + 4 * a.CB);                                    // [CB]
    const int cblk = bid % a.n_cblk, rest = bid / a.n_cblk;
    const int R0 = (rest % a.n_rt) * a.TR, C0 = (rest / a.n_rt) * a.TC;
    const int tid = threadIdx.x;
    {
        const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
        const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
        for (int e = tid; e < 4 * a.CB; e += 256) {
            const int k = e >> 2, side = e & 3;
            const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;   // o_i, i = side
            const int c = cblk * a.CB + k;
            int par = -1;
            T inv = 0;
            if (c < a.gxc * a.gyc) {
                const int cb = c / a.gxc, ca = c - cb * a.gxc;
                const int pb = parent_index(a.l, cb, sy), pa = parent_index(a.l, ca, sx);
                if (pb >= 0 && pb < a.gyp && pa >= 0 && pa < a.gxp && vxp[pa] && vyp[pb]) {
                    par = pb * a.gxp + pa;
                    int nx = 0, ny = 0;
                    for (int s2 = -1; s2 <= 1; s2 += 2) {
                        const int ccx = child_index(a.l, pa, s2), ccy = child_index(a.l, pb, s2);
                        nx += ccx >= 0 && ccx < a.gxc && vxc[ccx];
                        ny += ccy >= 0 && ccy < a.gyc && vyc[ccy];
                    }
                    inv = T(1) / T(nx * ny);
                }
                if (side == 0) sCv[k] = vxc[ca] && vyc[cb];
            } else if (side == 0) {
                sCv[k] = -1;   // past the last child: nothing to write
            }
            sPar[e] = par;
            sInv[e] = inv;
        }
    }
    __syncthreads();
    // Stage the parents' data.
    for (int e = tid; e < 4 * a.CB * per_side; e += 256) {
        const int ks = a.is_top ? (int)fdiv(e, a.f_t) : (int)fdiv(e, a.f_nr);
        const int rem = e - ks * per_side;
        const int side = ks & 3;
        const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;
        const int par = sPar[ks];
        T v = 0;
        uint8_t m = 255;
        if (par >= 0) {
            if (a.is_top) {
                const int ty = fdiv(rem, a.f_tc);
                const int qy = R0 + ty - sy, qx = C0 + rem - ty * a.TC - sx;
                if (qy >= 0 && qy < a.h && qx >= 0 && qx < a.w) {
                    const size_t o = ((size_t)par * a.h + qy) * a.w + qx;
                    v = dtop[o] * rect_grad_factor(top[o], lam);
                }
            } else {
                const int rr = fdiv(rem, a.f_rwd);
                const int ry = ((R0 - sy) >> 1) + rr, rx = ((C0 - sx) >> 1) + rem - rr * RWd;
                if (ry >= 0 && ry < a.hu && rx >= 0 && rx < a.wu) {
                    const size_t o = ((size_t)par * a.hu + ry) * a.wu + rx;
                    v = gp_cur[o];
                    m = code_cur[o];
                }
            }
        }
        sG[e] = v;
        if (!a.is_top) sM[e] = m;
    }
    __syncthreads();
    // g'_{l-1}(c, r) = lambda C'^((lambda-1)/lambda) * sum_i G_l(P_i, r - o_i) / |V(P_i)|
    for (int e = tid; e < a.CB * T_; e += 256) {
        const int k = fdiv(e, a.f_t), rem = e - k * T_;
        const int ty = fdiv(rem, a.f_tc), tx = rem - ty * a.TC;
        const int ry = R0 + ty, rx = C0 + tx;
        if (ry >= a.h || rx >= a.w || sCv[k] < 0) continue;
        const size_t o = (((size_t)cblk * a.CB + k) * a.h + ry) * a.w + rx;
        if (!sCv[k]) {
            gp_prev[o] = T(0);
            continue;
        }
        T acc = 0;
#pragma unroll
        for (int side = 0; side < 4; ++side) {
            const int ks = k * 4 + side;
            if (sPar[ks] < 0) continue;
            const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;
            const int qy = ry - sy, qx = rx - sx;
            if (qy < 0 || qy >= a.h || qx < 0 || qx >= a.w) continue;
            T gsum = 0;
            if (a.is_top) {
                gsum = sG[ks * per_side + rem];
            } else {
                const int ry0 = (R0 - sy) >> 1, rx0 = (C0 - sx) >> 1;
                for (int py = (qy - 1) >> 1; py <= (qy + 1) >> 1; ++py) {
                    const int my = qy - 2 * py;
                    if (my < -1 || my > 1) continue;
                    for (int px = (qx - 1) >> 1; px <= (qx + 1) >> 1; ++px) {
                        const int mx = qx - 2 * px;
                        if (mx < -1 || mx > 1) continue;
                        const int li = ks * per_side + (py - ry0) * RWd + (px - rx0);
                        if (sM[li] == 3 * (my + 1) + (mx + 1)) gsum += sG[li];
                    }
                }
            }
            acc += gsum * sInv[ks];
        }
        gp_prev[o] = acc * rect_grad_factor(cp_prev[o], lam);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd_level(BwdArgs a, const T* __restrict__ dtop, const T* __restrict__ top,
                                                   const T* __restrict__ gp_cur, const uint8_t* __restrict__ code_cur,
                                                   const T* __restrict__ cp_prev, const uint8_t* __restrict__ vt,
                                                   Geom g, T lam, T* __restrict__ gp_prev, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    bwd_level_body<T>(a, dtop, top, gp_cur, code_cur, cp_prev, vt, g, lam, gp_prev, bid);
}

struct BwdLevelJob {
    BwdArgs a;
    const float *dtop, *top, *gp_cur;
    const uint8_t* code_cur;
    const float* cp_prev;
    const uint8_t* vt;
    Geom g;
    float lam;
    float* gp_prev;
    static __device__ void run(const BwdLevelJob& j, int v) {
        bwd_level_body<float>(j.a, j.dtop, j.top, j.gp_cur, j.code_cur, j.cp_prev, j.vt, j.g, j.lam, j.gp_prev, v);
    }
};

// Gradient of L = sum over top patches P of max_q C_top(P, q): 1 at the first
// maximum of each top map (lowest index), 0 elsewhere.  One block per patch.
__device__ inline void top_grad_body(const float* __restrict__ top, int hw, float* __restrict__ dtop, int P) {
    __shared__ float sv[4];
    __shared__ int si[4];
    const float* m = top + (size_t)P * hw;
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int q = threadIdx.x; q < hw; q += 256) {
        const float v = m[q];
        if (v > bv) { bv = v; bi = q; }   // q increases: the first maximum of this thread's share
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const float ov = __shfl_xor(bv, d);
        const int oi = __shfl_xor(bi, d);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sv[wave] = bv; si[wave] = bi; }
    __syncthreads();
    bv = sv[0];
    bi = si[0];
    for (int w = 1; w < 4; ++w)
        if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) { bv = sv[w]; bi = si[w]; }
    for (int q = threadIdx.x; q < hw; q += 256) dtop[(size_t)P * hw + q] = q == bi ? 1.f : 0.f;
}

struct TopGradJob {
    const float* top;
    int hw;
    float* dtop;
    static __device__ void run(const TopGradJob& j, int v) { top_grad_body(j.top, j.hw, j.dtop, v); }
};

BwdArgs make_bwd_args(int l, const Geom& g, int& nblocks, size_t& smem) {
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
    a.TC = a.w < 128 ? a.w : 128;
    a.TR = 1024 / a.TC;
    if (a.TR > a.h) a.TR = a.h;
    if (a.TR < 1) a.TR = 1;
    a.CB = 1024 / (a.TR * a.TC);
    if (a.CB < 1) a.CB = 1;
    if (a.CB > 64) a.CB = 64;
    const int nc = a.gxc * a.gyc;
    a.n_cblk = (nc + a.CB - 1) / a.CB;
    a.n_rt = (a.h + a.TR - 1) / a.TR;
    const int n_ct = (a.w + a.TC - 1) / a.TC;
    const int RH = a.TR / 2 + 2, RWd = a.TC / 2 + 2;
    a.f_t = make_fastdiv(a.TR * a.TC);
    a.f_tc = make_fastdiv(a.TC);
    a.f_nr = make_fastdiv(RH * RWd);
    a.f_rwd = make_fastdiv(RWd);
    const int per_side = a.is_top ? a.TR * a.TC : RH * RWd;
    smem = (size_t)4 * a.CB * per_side * (sizeof(float) + 1);
    smem = (smem + 15) & ~size_t(15);
    smem += (size_t)4 * a.CB * (sizeof(int) + sizeof(double)) + (size_t)a.CB * sizeof(int) + 16;
    nblocks = a.n_cblk * a.n_rt * n_ct;
    return a;
}

}  // namespace

JobRec bwd_level_job(int l, const float* dtop, const float* top, const float* gp_cur, const uint8_t* code_cur,
                     const float* cp_prev, const uint8_t* vt, const Geom& g, float lam, float* gp_prev) {
    int nb;
    size_t smem;
    const BwdArgs a = make_bwd_args(l, g, nb, smem);
    JobRec r;
    r.set(JK_BWD_LEVEL, nb, smem, BwdLevelJob{a, dtop, top, gp_cur, code_cur, cp_prev, vt, g, lam, gp_prev});
    return r;
}

JobRec top_grad_job(const float* top, const Geom& g, float* dtop) {
    JobRec r;
    const int lt = g.lmax;
    r.set(JK_TOP_GRAD, g.gx[lt] * g.gy[lt], 0, TopGradJob{top, g.h[lt] * g.w[lt], dtop});
    return r;
}

hipError_t launch_group_bwd(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_BWD_LEVEL: return launch_grouped<BwdLevelJob, 256, 1>(gl, s);
        case JK_TOP_GRAD: return launch_grouped<TopGradJob, 256, 1>(gl, s);
        default: return hipErrorInvalidValue;
    }
}

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
    a.TC = a.w < 128 ? a.w : 128;
    a.TR = 1024 / a.TC;
    if (a.TR > a.h) a.TR = a.h;
    if (a.TR < 1) a.TR = 1;
    a.CB = 1024 / (a.TR * a.TC);
    if (a.CB < 1) a.CB = 1;
    if (a.CB > 64) a.CB = 64;
    const int nc = a.gxc * a.gyc;
    a.n_cblk = (nc + a.CB - 1) / a.CB;
    a.n_rt = (a.h + a.TR - 1) / a.TR;
    const int n_ct = (a.w + a.TC - 1) / a.TC;
    const int RH = a.TR / 2 + 2, RWd = a.TC / 2 + 2;
    a.f_t = make_fastdiv(a.TR * a.TC);
    a.f_tc = make_fastdiv(a.TC);
    a.f_nr = make_fastdiv(RH * RWd);
    a.f_rwd = make_fastdiv(RWd);
    const int per_side = a.is_top ? a.TR * a.TC : RH * RWd;
    size_t smem = (size_t)4 * a.CB * per_side * (sizeof(T) + 1);
    smem = (smem + 15) & ~size_t(15);
    smem += (size_t)4 * a.CB * (sizeof(int) + sizeof(T)) + (size_t)a.CB * sizeof(int) + 16;
    const int nblocks = a.n_cblk * a.n_rt * n_ct;
    hipLaunchKernelGGL(k_bwd_level<T>, dim3(((nblocks + 7) / 8) * 8), dim3(256), smem, s, a, dtop, top, gp_cur,
                       code_cur, cp_prev, vt, g, lam, gp_prev, nblocks);
    return hipGetLastError();
}

template hipError_t launch_bwd_level<float>(int, const float*, const float*, const float*, const uint8_t*,
                                            const float*, const uint8_t*, const Geom&, float, float*, hipStream_t);
template hipError_t launch_bwd_level<double>(int, const double*, const double*, const double*, const uint8_t*,
                                             const double*, const uint8_t*, const Geom&, double, double*,
                                             hipStream_t);

}  // namespace dm
