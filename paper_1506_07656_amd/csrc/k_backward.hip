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
#include <type_traits>

#include "dm_group.h"

namespace dm {
namespace {

template <typename T>
__device__ inline T rect_grad_factor(T c, T lam) {
    // d(max(A,0)^lam)/dA written from the stored value c = A^lam.
    return c > T(0) ? lam * rect_pow(c, (lam - T(1)) / lam) : T(0);
}

// A gradient entry as FP32, or rounded to BF16 (nearest even) when the
// array holds BF16.
template <typename T>
__device__ inline void store_grad(T* p, size_t i, T v, int as_bf16) {
    if (std::is_same<T, float>::value && as_bf16) {
        uint32_t u = __float_as_uint((float)v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        reinterpret_cast<uint16_t*>(p)[i] = (uint16_t)(u >> 16);
    } else {
        p[i] = v;
    }
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
    int out16;                        // the output gradient is stored as BF16 (FP32 path only)
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
            store_grad(gp_prev, o, T(0), a.out16);
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
        store_grad(gp_prev, o, acc * rect_grad_factor(cp_prev[o], lam), a.out16);
    }
}

// Row-streaming form of the level adjoint below the top (FP32, child maps at
// least 32 columns wide).  One wave owns a child c, a band of rows and 64
// output columns (one per lane).  Step rp brings pooled row rp of each
// parent's g'_l and codes (lanes 0..33 cover the pooled columns the wave's
// outputs can receive from) and adds every entry, times 1/|V(P_i)|, to the
// output it reaches, r = 2r' + m + o_i, in a 6-row ring of output sums in
// LDS.  Entries of one row are added in two passes (even pooled columns,
// then odd ones), so that no two lanes of a pass touch one sum: every sum
// is formed in a fixed order (step, side, pass) and the result is
// deterministic.  U_l row r' is the last to reach output rows <= 2r' - 1,
// so after step rp the rows 2rp-2, 2rp-1 are final: they are taken out of
// the ring (cleared for reuse) and C'_{l-1} is read only where the sum is
// non-zero (an out-of-range offset elsewhere), one step ahead of the
// multiply by the rectification factor.  Only window outputs are added to,
// so every added sum is taken exactly once.
constexpr int kBwCols = 64;
constexpr int kBwWaves = 4;
constexpr int kBwRing = 8;     // live output rows 2r'-2 .. 2r'+2 (5), rounded up to a power of two
constexpr int kOOB = 0x7ffffff0;   // buffer byte offset past any map

struct BwStreamArgs {
    int l;
    int gxp, gyp, gxc, gyc;
    int h, w;      // child pooled grid (maps of level l)
    int hu, wu;    // pooled grid of level l
    int TR, n_band, n_ct, n_cgrp;
    int out16;     // the output gradient is stored as BF16 (level 1 feeding the BF16 bottom)
};

// Window offsets of an argmax code k = 3 m_y + m_x (m in 0..2): 2-bit fields
// of two constants, read with one bit-field extract each.
__device__ inline int code_my(int k) { return (0x2A540u >> (2 * k)) & 3u; }
__device__ inline int code_mx(int k) { return (0x24924u >> (2 * k)) & 3u; }

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, nbytes, 0x00020000);
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void bwd_level_stream_body(const BwStreamArgs& a, const float* __restrict__ gp_cur,
                                             const uint8_t* __restrict__ code_cur, const float* __restrict__ cp_prev,
                                             const uint8_t* __restrict__ vt, const Geom& g, float lam,
                                             float* __restrict__ gp_prev, int bid) {
    constexpr int NPX = kBwCols / 2 + 2;
    __shared__ float sR[kBwWaves][kBwRing][kBwCols];
    const int cgrp = bid % a.n_cgrp, rest = bid / a.n_cgrp;
    const int ct = rest % a.n_ct, band = rest / a.n_ct;
    const int t = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index: uniform
    const int R0 = band * a.TR, R1 = min(R0 + a.TR, a.h);
    const int C0 = ct * kBwCols, Cend = min(C0 + kBwCols, a.w);
    const int c = cgrp * kBwWaves + wv;
    if (c >= a.gxc * a.gyc) return;
    const int cb = c / a.gxc, ca = c - cb * a.gxc;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    const int rx = C0 + t;
    const bool lane_o = rx < Cend;
    const size_t obase = (size_t)c * a.h * a.w;
    if (!(vxc[ca] && vyc[cb])) {   // no child here: its gradient is 0
        for (int ry = R0; ry < R1; ++ry)
            if (lane_o) store_grad(gp_prev, obase + (size_t)ry * a.w + rx, 0.f, a.out16);
        return;
    }
    const int usz = a.hu * a.wu, nparent = a.gxp * a.gyp;
    const __amdgpu_buffer_rsrc_t rsG = rsrc(gp_cur, nparent * usz * 4), rsM = rsrc(code_cur, nparent * usz);
    const __amdgpu_buffer_rsrc_t rsC = rsrc(cp_prev, a.gxc * a.gyc * a.h * a.w * 4);
    // Element offset of each parent's map, or a large negative value for a
    // missing parent: with a lane's row offset added (also large negative
    // when the lane or row has no entry), an entry exists exactly when the
    // sum is >= 0, so validity needs no lane masks per side.
    constexpr int kNone = -(1 << 30);
    int pbase[4];
    float inv[4];
#pragma unroll
    for (int side = 0; side < 4; ++side) {
        const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;   // o_i, i = side
        const int pb = parent_index(a.l, cb, sy), pa = parent_index(a.l, ca, sx);
        const bool ok = pb >= 0 && pb < a.gyp && pa >= 0 && pa < a.gxp && vxp[pa] && vyp[pb];
        pbase[side] = ok ? (pb * a.gxp + pa) * usz : kNone;
        int nx = 0, ny = 0;
        if (ok) {
            for (int s2 = -1; s2 <= 1; s2 += 2) {
                const int ccx = child_index(a.l, pa, s2), ccy = child_index(a.l, pb, s2);
                nx += ccx >= 0 && ccx < a.gxc && vxc[ccx];
                ny += ccy >= 0 && ccy < a.gyc && vyc[ccy];
            }
        }
        inv[side] = ok ? 1.f / float(nx * ny) : 0.f;
    }
    float (*ring)[kBwCols] = sR[wv];
    for (int e = t; e < kBwRing * kBwCols; e += 64) (&ring[0][0])[e] = 0.f;
    wave_sync();
    const int ux = (C0 >> 1) - 1 + t;          // the lane's pooled column while adding
    const bool lane_u = t < NPX && ux >= 0 && ux < a.wu;
    struct RowBuf { float g[4]; int m[4]; };
    struct OutBuf { float acc[2]; float cv[2]; };
    auto load_row = [&](int rp, RowBuf& b) {
        const bool rok = lane_u && rp >= 0 && rp < a.hu;
        const int roff = rok ? rp * a.wu + ux : kNone;
#pragma unroll
        for (int side = 0; side < 4; ++side) {
            const int off = pbase[side] + roff;   // >= 0 exactly for an existing entry
            const bool ok = off >= 0;
            const float v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsG, ok ? off * 4 : kOOB, 0, 0));
            const int m = __builtin_amdgcn_raw_buffer_load_b8(rsM, ok ? off : kOOB, 0, 0);
            b.g[side] = ok ? v : 0.f;
            b.m[side] = m;
        }
    };
    auto add_row = [&](int rp, const RowBuf& b) {
#pragma unroll
        for (int side = 0; side < 4; ++side) {
            if (pbase[side] < 0) continue;   // uniform: no parent on this side
            const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;
            const int ry = 2 * rp + code_my(b.m[side]) - 1 + sy, rxx = 2 * ux + code_mx(b.m[side]) - 1 + sx;
            const bool hit = b.g[side] != 0.f && (unsigned)(ry - R0) < (unsigned)(R1 - R0) &&
                             (unsigned)(rxx - C0) < (unsigned)(Cend - C0);
            // Within one instruction no two lanes of the same column parity
            // meet on a position, so an LDS add without return is exactly
            // old + v; the even pass precedes the odd one (a wave's LDS
            // operations run in order), which fixes the order of every sum.
#pragma unroll
            for (int pass = 0; pass < 2; ++pass)
                if (hit && (ux & 1) == pass) atomicAdd(&ring[ry & (kBwRing - 1)][rxx - C0], b.g[side] * inv[side]);
        }
    };
    auto collect = [&](int rp, OutBuf& o) {
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int ry = 2 * rp - 2 + dy;
            float acc = 0.f;
            if (ry >= R0 && ry < R1 && lane_o) {
                acc = ring[ry & (kBwRing - 1)][t];
                ring[ry & (kBwRing - 1)][t] = 0.f;
            }
            o.acc[dy] = acc;
            const int off = ry * a.w + rx;   // used only where acc != 0
            o.cv[dy] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                rsC, acc != 0.f ? (int)(obase + off) * 4 : kOOB, 0, 0));
        }
    };
    auto finish = [&](int rp, const OutBuf& o) {
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int ry = 2 * rp - 2 + dy;
            if (ry < R0 || ry >= R1 || !lane_o) continue;
            store_grad(gp_prev, obase + (size_t)ry * a.w + rx, o.acc[dy] * rect_grad_factor(o.cv[dy], lam), a.out16);
        }
    };
    const int rpa = (R0 - 2) >> 1, rp1 = ((R1 - 1) >> 1) + 1;
    RowBuf b0, b1;
    OutBuf o0, o1;
    o1.acc[0] = o1.acc[1] = 0.f;
    o1.cv[0] = o1.cv[1] = 0.f;
    load_row(rpa, b0);
    int rp = rpa;
    for (;;) {
        load_row(rp + 1, b1);
        add_row(rp, b0);
        collect(rp, o0);
        finish(rp - 1, o1);
        wave_sync();
        if (rp == rp1) {
            finish(rp, o0);
            break;
        }
        ++rp;
        load_row(rp + 1, b0);
        add_row(rp, b1);
        collect(rp, o1);
        finish(rp - 1, o0);
        wave_sync();
        if (rp == rp1) {
            finish(rp, o1);
            break;
        }
        ++rp;
    }
}

__global__ __launch_bounds__(64 * kBwWaves) void k_bwd_level_stream(BwStreamArgs a, const float* __restrict__ gp_cur,
                                                                     const uint8_t* __restrict__ code_cur,
                                                                     const float* __restrict__ cp_prev,
                                                                     const uint8_t* __restrict__ vt, Geom g, float lam,
                                                                     float* __restrict__ gp_prev, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    bwd_level_stream_body(a, gp_cur, code_cur, cp_prev, vt, g, lam, gp_prev, bid);
}

struct BwdLevelStreamJob {
    BwStreamArgs a;
    const float* gp_cur;
    const uint8_t* code_cur;
    const float* cp_prev;
    const uint8_t* vt;
    Geom g;
    float lam;
    float* gp_prev;
    static __device__ void run(const BwdLevelStreamJob& j, int v) {
        bwd_level_stream_body(j.a, j.gp_cur, j.code_cur, j.cp_prev, j.vt, j.g, j.lam, j.gp_prev, v);
    }
};

// The streaming form serves FP32 steps below the top whose child maps are at
// least 32 columns wide and whose arrays stay below 2^31 bytes.
bool use_bwd_stream(int l, const Geom& g) {
    if (l == g.lmax || g.w[l] < 32) return false;
    return (double)g.gx[l] * g.gy[l] * g.h[l + 1] * g.w[l + 1] * 4 < 2.0e9 &&
           (double)g.gx[l - 1] * g.gy[l - 1] * g.h[l] * g.w[l] * 4 < 2.0e9;
}

BwStreamArgs make_bwd_stream_args(int l, const Geom& g, int& nblocks) {
    BwStreamArgs b;
    b.out16 = 0;
    b.l = l;
    b.gxp = g.gx[l];
    b.gyp = g.gy[l];
    b.gxc = g.gx[l - 1];
    b.gyc = g.gy[l - 1];
    b.h = g.h[l];
    b.w = g.w[l];
    b.hu = g.h[l + 1];
    b.wu = g.w[l + 1];
    b.TR = b.h < 64 ? ((b.h + 1) & ~1) : 64;
    b.n_band = (b.h + b.TR - 1) / b.TR;
    b.n_ct = (b.w + kBwCols - 1) / kBwCols;
    b.n_cgrp = (b.gxc * b.gyc + kBwWaves - 1) / kBwWaves;
    nblocks = b.n_cgrp * b.n_ct * b.n_band;
    return b;
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
    a.out16 = 0;
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
                     const float* cp_prev, const uint8_t* vt, const Geom& g, float lam, float* gp_prev, bool out16) {
    int nb;
    if (use_bwd_stream(l, g)) {
        BwStreamArgs b = make_bwd_stream_args(l, g, nb);
        b.out16 = out16;
        JobRec r;
        r.set(JK_BWD_LEVEL_STREAM, nb, 0, BwdLevelStreamJob{b, gp_cur, code_cur, cp_prev, vt, g, lam, gp_prev});
        return r;
    }
    size_t smem;
    BwdArgs a = make_bwd_args(l, g, nb, smem);
    a.out16 = out16;
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
        case JK_BWD_LEVEL_STREAM: return launch_grouped<BwdLevelStreamJob, 64 * kBwWaves, 1>(gl, s);
        case JK_TOP_GRAD: return launch_grouped<TopGradJob, 256, 1>(gl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_bwd_level(int l, const T* dtop, const T* top, const T* gp_cur, const uint8_t* code_cur,
                            const T* cp_prev, const uint8_t* vt, const Geom& g, T lam, T* gp_prev, hipStream_t s,
                            bool out16) {
    if constexpr (std::is_same<T, float>::value) {
        if (use_bwd_stream(l, g)) {
            int nb;
            BwStreamArgs b = make_bwd_stream_args(l, g, nb);
            b.out16 = out16;
            hipLaunchKernelGGL(k_bwd_level_stream, dim3(((nb + 7) / 8) * 8), dim3(64 * kBwWaves), 0, s, b, gp_cur,
                               code_cur, cp_prev, vt, g, lam, gp_prev, nb);
            return hipGetLastError();
        }
    }
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
    a.out16 = out16;
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
                                            const float*, const uint8_t*, const Geom&, float, float*, hipStream_t,
                                            bool);
template hipError_t launch_bwd_level<double>(int, const double*, const double*, const double*, const uint8_t*,
                                             const double*, const uint8_t*, const Geom&, double, double*,
                                             hipStream_t, bool);

}  // namespace dm
