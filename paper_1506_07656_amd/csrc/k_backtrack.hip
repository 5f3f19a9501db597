// Top-down correspondence extraction (Sec. 3.3, Eqs. (13)-(16)).
//
// The paper expands tuples (N, p, p', s) with B (Eq. (14)) from every
// top-level entry and, whenever two tuples share (N, p, p'), keeps the higher
// score.  Since the subtree below a tuple depends only on (N, p, p'), this is
// the max-plus recursion, evaluated here densely level by level as a gather:
//
//   V_l(P, q)   best score of a tuple reaching node (l, P, q);  V_top = C_top
//   U_{l-1}(c, r) = C'_{l-1}(c, r) + max_{i: P = c - 2^l o_i exists} V_l(P, r - o_i)
//   V_{l-1}(c, x) = max { U_{l-1}(c, r) : 2r + m_{l-1}(c, r) = x }        (Eq. (13))
//
// U lives on the pooled grid (a quarter of V's), so only U and the argmax
// codes are stored.  At the bottom U_0 is not written: each (c, r) gives the
// atomic tuple (c, x = 2r + m, U_0) of M' (Eq. (15)), which is folded into
// two tables of packed keys (score bits << 32 | inverted tie-break index):
//   best[c]     BestAt(p):   max score, ties to the smallest (x'_y, x'_x)
//   cell[c']    BestAt'(p'): max score over the 4x4 target cell, ties to the
//               smallest (p_y, p_x, p'_y, p'_x)
// Scores are sums of non-negative values, so their float bits order like the
// floats and the packed 64-bit maxima are exact and order independent.
#include "dm_group.h"

namespace dm {
namespace {

// Non-negative float <-> order-preserving code with 0 = "no tuple".
__device__ inline uint32_t enc(float v) { return __float_as_uint(v) + 1u; }
__device__ inline float dec(uint32_t e) { return __uint_as_float(e - 1u); }

struct BtArgs {
    int l;                       // the step reads level l and produces level l-1
    int gxp, gyp, gxc, gyc;      // parent (level l) and child (level l-1) lattices
    int h, w;                    // child pooled grid = maps of level l (h_l x w_l)
    int hu, wu;                  // U_l grid (h_{l+1} x w_{l+1}); unused at the top
    int is_top, is_bottom;
    int TR, TC, CB;              // tile rows, cols, children per block
    int n_cblk, n_rt;
    int cy0, cx0, ncy, ncx;      // cell-table window parameters (bottom only)
    int W2, cw;                  // target width, cells per target row
    FastDiv f_t, f_tc, f_nr, f_rwd;   // divisions by TR*TC, TC, RH*RWd, RWd (element indices < 2^14)
};

__device__ inline int xcd_block(int nblocks) {
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Local maximum of a map (DM* entry points): positive, not below any 3 x 3
// neighbour inside the h x w map, above the neighbours before it in raster
// order (one maximum per plateau).
__device__ inline bool local_max(const float* __restrict__ m, int h, int w, int y, int x) {
    const float v = m[(size_t)y * w + x];
    if (!(v > 0.f)) return false;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int yy = y + dy, xx = x + dx;
            if ((dy == 0 && dx == 0) || yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
            const float n = m[(size_t)yy * w + xx];
            if (dy < 0 || (dy == 0 && dx < 0) ? !(v > n) : !(v >= n)) return false;
        }
    return true;
}

constexpr uint8_t kEntryBit = 0x10;   // DM*: the pooled cell is an entry point (above the 4-bit code)

// RECT: a run of invariant matching; the bottom step maps each tuple back to
// the input images and reduces into the tables shared by all runs.
// DMSTAR: entry points at the local maxima of every level (codes carry
// kEntryBit): a top position enters only at a local maximum, and a pooled
// cell marked as an entry starts a tuple with its own value.  DMSTAR = 1
// scores by path sums: where a tuple arrives from above it scores at least as
// much as the entry, so the entry counts only where none arrives.
// DMSTAR = 2 scores by the start and end of each path: above the bottom a
// node keeps the larger of the arriving start value and its own value if it
// is an entry, and the bottom step adds the atomic value (as for path sums,
// so the bottom step is the same code for both).
template <bool RECT, int DMSTAR = 0>
__device__ inline void bt_body(const BtArgs& a, const float* __restrict__ cp_prev,
                               const uint8_t* __restrict__ code_prev, const float* __restrict__ u_cur,
                               const uint8_t* __restrict__ code_cur, const float* __restrict__ top,
                               const uint8_t* __restrict__ vt, const Geom& g, float* __restrict__ u_prev,
                               unsigned long long* __restrict__ best, unsigned long long* __restrict__ cell, int bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = a.TR * a.TC;
    uint32_t* sV = (uint32_t*)smem_raw;                                   // [CB][4][TR][TC]
    unsigned long long* sBest = (unsigned long long*)(sV + 4 * a.CB * T);  // [CB]
    unsigned long long* sCell = sBest + a.CB;                               // [ncy][ncx]
    int* sPar = (int*)(sCell + a.ncy * a.ncx);                              // [CB][4] parent map index
    int* sCv = sPar + 4 * a.CB;                                             // [CB] child exists
    const int cblk = bid % a.n_cblk, rest = bid / a.n_cblk;   // once per block (scalar)
    const int R0 = (rest % a.n_rt) * a.TR, C0 = (rest / a.n_rt) * a.TC;
    const int tid = threadIdx.x;
    {
        const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
        const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
        for (int e = tid; e < 4 * a.CB; e += 256) {
            const int k = e >> 2, side = e & 3;
            const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;  // o_i of Eq. (5), i = side
            const int c = cblk * a.CB + k;
            int par = -1;
            if (c < a.gxc * a.gyc) {
                const int cb = c / a.gxc, ca = c - cb * a.gxc;
                const int pb = parent_index(a.l, cb, sy), pa = parent_index(a.l, ca, sx);
                if (pb >= 0 && pb < a.gyp && pa >= 0 && pa < a.gxp && vxp[pa] && vyp[pb]) par = pb * a.gxp + pa;
                if (side == 0) sCv[k] = vxc[ca] && vyc[cb];
            } else if (side == 0) {
                sCv[k] = 0;
            }
            sPar[e] = par;
        }
        if (a.is_bottom) {
            for (int e = tid; e < a.CB; e += 256) sBest[e] = 0ull;
            for (int e = tid; e < a.ncy * a.ncx; e += 256) sCell[e] = 0ull;
        }
        if (!a.is_top)
            for (int e = tid; e < 4 * a.CB * T; e += 256) sV[e] = 0u;
    }
    __syncthreads();

    // Phase 1: V_l of the up-to-4 parents of each child, on the shifted tile.
    if (a.is_top) {
        for (int e0 = tid; e0 < 4 * a.CB * T; e0 += 4 * 256) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * 256;
                v[u] = 0u;
                if (e < 4 * a.CB * T) {
                    const int ks = fdiv(e, a.f_t), rem = e - ks * T;
                    const int side = ks & 3;
                    const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;
                    const int par = sPar[ks];
                    const int ty = fdiv(rem, a.f_tc);
                    const int qy = R0 + ty - sy, qx = C0 + rem - ty * a.TC - sx;
                    if (par >= 0 && qy >= 0 && qy < a.h && qx >= 0 && qx < a.w &&
                        (!DMSTAR || local_max(top + (size_t)par * a.h * a.w, a.h, a.w, qy, qx)))
                        v[u] = enc(top[((size_t)par * a.h + qy) * a.w + qx]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + u * 256 < 4 * a.CB * T) sV[e0 + u * 256] = v[u];
        }
    } else {
        // U_l entries r' whose argmax 2r' + m can land in this side's q-range
        // [q0, q0 + TR): r' in [floor(q0/2), floor((q0 + TR)/2)].
        const int RH = a.TR / 2 + 2, RWd = a.TC / 2 + 2, NR = RH * RWd;
        for (int e0 = tid; e0 < 4 * a.CB * NR; e0 += 2 * 256) {
            float uv[2];
            int m[2], idx[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = e0 + u * 256;
                idx[u] = -1;
                uv[u] = -1.f;
                m[u] = 0;
                if (e >= 4 * a.CB * NR) continue;
                const int ks = fdiv(e, a.f_nr), rem = e - ks * NR;
                const int par = sPar[ks];
                if (par < 0) continue;
                const int side = ks & 3;
                const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;
                const int qy0 = R0 - sy, qx0 = C0 - sx;
                const int rr = fdiv(rem, a.f_rwd);
                const int ry = (qy0 >> 1) + rr, rx = (qx0 >> 1) + rem - rr * RWd;   // >> 1: floor division
                if (ry > ((qy0 + a.TR) >> 1) || rx > ((qx0 + a.TC) >> 1)) continue;
                if (ry < 0 || ry >= a.hu || rx < 0 || rx >= a.wu) continue;
                const size_t o = ((size_t)par * a.hu + ry) * a.wu + rx;
                uv[u] = u_cur[o];
                m[u] = code_cur[o] & (DMSTAR ? 15 : 255);
                const int qy = 2 * ry + m[u] / 3 - 1, qx = 2 * rx + m[u] % 3 - 1;
                const int ty = qy - qy0, tx = qx - qx0;   // tile index of r = q + o_i
                if (ty >= 0 && ty < a.TR && tx >= 0 && tx < a.TC) idx[u] = (ks * a.TR + ty) * a.TC + tx;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (idx[u] >= 0 && uv[u] >= 0.f) atomicMax(&sV[idx[u]], enc(uv[u]));   // unreached: -inf
        }
    }
    __syncthreads();

    // Phase 2: U_{l-1}(c, r) = C'_{l-1}(c, r) + max over parents.
    const int cyb = (2 * R0 - 1) >> 2, cxb = (2 * C0 - 1) >> 2;   // floor division by 4
    for (int e0 = tid; e0 < a.CB * T; e0 += 4 * 256) {
        float cpv[4];
        int mv[4];
        uint32_t vb[4];
        size_t off[4];
        bool live[4], ent[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {   // loads of 4 entries first, so they overlap
            const int e = e0 + u * 256;
            live[u] = false;
            ent[u] = false;
            vb[u] = 0u;
            cpv[u] = 0.f;
            mv[u] = 0;
            off[u] = 0;
            if (e >= a.CB * T) continue;
            const int k = fdiv(e, a.f_t), rem = e - k * T;
            const int ty = fdiv(rem, a.f_tc), tx = rem - ty * a.TC;
            const int ry = R0 + ty, rx = C0 + tx;
            if (!sCv[k] || ry >= a.h || rx >= a.w) continue;
            live[u] = true;
#pragma unroll
            for (int side = 0; side < 4; ++side) vb[u] = max(vb[u], sV[((k * 4 + side) * a.TR + ty) * a.TC + tx]);
            off[u] = ((size_t)child_slot(g, a.l, cblk * a.CB + k) * a.h + ry) * a.w + rx;
            if constexpr (DMSTAR != 0) {
                const int cm = code_prev[off[u]];
                ent[u] = (cm & kEntryBit) != 0;
                mv[u] = cm & 15;
                if (vb[u] || ent[u] || !a.is_bottom) cpv[u] = cp_prev[off[u]];
            } else if (vb[u] || !a.is_bottom) {
                cpv[u] = cp_prev[off[u]];
                if (a.is_bottom) mv[u] = code_prev[off[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!live[u]) continue;
            const uint32_t arrived = vb[u];
            if (ent[u] && !vb[u]) vb[u] = enc(0.f);   // an entry with nothing above: its own value
            if (!a.is_bottom) {
                if constexpr (DMSTAR == 2)   // start/end scores: the start value passes down unchanged
                    u_prev[off[u]] = arrived ? (ent[u] ? fmaxf(dec(arrived), cpv[u]) : dec(arrived))
                                             : (ent[u] ? cpv[u] : -INFINITY);
                else
                    u_prev[off[u]] = vb[u] ? cpv[u] + dec(vb[u]) : -INFINITY;
                continue;
            }
            if (!vb[u]) continue;
            const int e = e0 + u * 256;
            const int k = fdiv(e, a.f_t), rem = e - k * T;
            const int ty = fdiv(rem, a.f_tc), tx = rem - ty * a.TC;
            const int c = cblk * a.CB + k, ry = R0 + ty, rx = C0 + tx;
            const float uu = cpv[u] + dec(vb[u]);
            const int xy = 2 * ry + mv[u] / 3 - 1, xx = 2 * rx + mv[u] % 3 - 1;
            const unsigned long long hi = (unsigned long long)__float_as_uint(uu) << 32;
            if constexpr (RECT) {
                int qx, qy, px, py;
                if (rect_target(g.rect, xx, xy, qx, qy)) {
                    rect_source(g.rect, c % a.gxc, c / a.gxc, px, py);
                    atomicMax(&sBest[k], hi | (0xFFFFFFFFull - (uint32_t)(qy * g.rect.W2o + qx)));
                    atomicMax(&cell[(size_t)(qy >> 2) * g.rect.cw2 + (qx >> 2)],
                              hi | (0xFFFFFFFFull - (uint32_t)((py * g.rect.W1o + px) * 16 + (qy & 3) * 4 + (qx & 3))));
                }
            } else {
                atomicMax(&sBest[k], hi | (0xFFFFFFFFull - (uint32_t)(xy * a.W2 + xx)));
                const unsigned long long kc = hi | (0xFFFFFFFFull - (uint32_t)(c * 16 + (xy & 3) * 4 + (xx & 3)));
                atomicMax(&sCell[((xy >> 2) - cyb) * a.ncx + ((xx >> 2) - cxb)], kc);
            }
        }
    }
    if (a.is_bottom) {
        __syncthreads();
        for (int e = tid; e < a.CB; e += 256) {
            const int c = cblk * a.CB + e;
            if (c < a.gxc * a.gyc && sBest[e]) {
                int slot = c;
                if constexpr (RECT) {
                    int px, py;
                    rect_source(g.rect, c % a.gxc, c / a.gxc, px, py);
                    slot = (py >> 2) * g.rect.cw1 + (px >> 2);
                }
                atomicMax(&best[slot], sBest[e]);
            }
        }
        for (int e = tid; e < a.ncy * a.ncx; e += 256) {
            const unsigned long long v = sCell[e];
            if (!v) continue;
            const int cy = cyb + e / a.ncx, cx = cxb + e % a.ncx;
            atomicMax(&cell[(size_t)cy * a.cw + cx], v);
        }
    }
}

// Row-streaming form of k_backtrack below the top, for child maps at least
// 32 columns wide.  One wave owns a child c, a band of TR rows of its pooled
// grid and 60 columns (one per lane; the parents' entries that can reach
// them span 32 columns, so each lane loads and scatters two of the four
// parents at once).  It walks down the rows of U_l of the
// child's (up to 4) parents.  Each U_l entry of parent P_i = c - 2^l o_i
// reaches V_l(P_i, x) at x = 2r' + m, hence the child's candidate at
// r = x + o_i, so the entry goes straight (max on collision, packed keys) into
// a small ring of candidate rows R(c, r) = max_i V_l(P_i, r - o_i) in LDS.
// U_l row r' is the last that can reach rows <= 2r', so after it the output
// rows 2r'-2, 2r'-1 are final: each entry is taken out of the ring with an
// exchange against 0 (so the ring is clean for its next row), and C'_{l-1}
// and its code are read only where a tuple arrived (lanes without one use an
// out-of-range buffer offset, which touches no memory).  Only window entries
// are scattered, so every scattered entry is taken exactly once.  Loads run
// one step ahead of their use.
// At the bottom the 4 waves of a block (4 children, same rows and columns)
// share the cell-table window; BestAt(c) is reduced within the wave.
constexpr int kBtCols = 64;    // lanes per wave: width of the candidate ring
// Output columns per wave: 60 (the parents' U_l entries that reach them span
// 32 columns, so the 64 lanes load and scatter two sides at once) or 64 (34
// columns: one side at a time, fewer waves when the map is 64 k wide).
constexpr int kBtWaves = 4;
constexpr int kBtRing = 8;     // live candidate rows 2r'-2 .. 2r'+2 (5), rounded up to a power of two
constexpr int kBtMaxTR = 64;   // tallest band (sizes the cell window in LDS)
constexpr int kBtTR = 64;      // band of the single-pair launch
constexpr int kOOB = 0x7ffffff0;   // buffer byte offset past any map (element offsets stay < 2^29)

struct BtStreamArgs {
    int l;
    int gxp, gyp, gxc, gyc;
    int h, w, hu, wu;
    int is_bottom;
    int TR, n_band, n_ct, n_cgrp;
    int W2, cw;
    int tile;   // output columns per wave (60 or 64)
};

// Window offsets of an argmax code k = 3 m_y + m_x (m in 0..2): 2-bit fields
// of two constants, read with one bit-field extract each.
__device__ inline int code_my(int k) { return (0x2A540u >> (2 * k)) & 3u; }
__device__ inline int code_mx(int k) { return (0x24924u >> (2 * k)) & 3u; }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Buffer descriptor over [p, p + nbytes): loads outside return 0.
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, nbytes, 0x00020000);
}

template <bool RECT, int TILE, bool BOTTOM, int DMSTAR = 0>
__device__ inline void bt_stream_body(const BtStreamArgs& a, const float* __restrict__ cp_prev,
                                      const uint8_t* __restrict__ code_prev, const float* __restrict__ u_cur,
                                      const uint8_t* __restrict__ code_cur, const uint8_t* __restrict__ vt,
                                      const Geom& g, float* __restrict__ u_prev,
                                      unsigned long long* __restrict__ best, unsigned long long* __restrict__ cell,
                                      int bid) {
    constexpr int NCX = kBtCols / 2 + 2;
    __shared__ uint32_t sR[kBtWaves][kBtRing][kBtCols];
    __shared__ unsigned long long sCell[(kBtMaxTR / 2 + 2) * NCX];
    const int cgrp = bid % a.n_cgrp, rest = bid / a.n_cgrp;
    const int ct = rest % a.n_ct, band = rest / a.n_ct;
    const int tid = threadIdx.x, t = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index: uniform
    const int R0 = band * a.TR, R1 = min(R0 + a.TR, a.h);
    const int C0 = ct * TILE, Cend = min(C0 + TILE, a.w);
    const int ncy = a.TR / 2 + 2;
    const int cyb = (2 * R0 - 1) >> 2, cxb = (2 * C0 - 1) >> 2;   // floor division by 4
    {
        uint32_t* flat = &sR[0][0][0];
        for (int e = tid; e < kBtWaves * kBtRing * kBtCols; e += 64 * kBtWaves) flat[e] = 0u;
        if constexpr (BOTTOM)
            for (int e = tid; e < ncy * NCX; e += 64 * kBtWaves) sCell[e] = 0ull;
    }
    __syncthreads();
    const int c = cgrp * kBtWaves + wv;
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    int cb = 0, ca = 0;
    bool live = c < a.gxc * a.gyc;
    if (live) {
        cb = c / a.gxc;
        ca = c - cb * a.gxc;
        live = vxc[ca] && vyc[cb];
    }
    unsigned long long mybest = 0ull;
    int pidx = 0, scell = c;   // invariant runs: the rectified source pixel and its cell
    if constexpr (RECT) {
        if (live) {
            int px, py;
            rect_source(g.rect, ca, cb, px, py);
            pidx = py * g.rect.W1o + px;
            scell = (py >> 2) * g.rect.cw1 + (px >> 2);
        }
    }
    if (live) {
        const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
        // One descriptor per parent array (below 2^31 bytes, checked at
        // launch; parents are selected by element offsets) and one over this
        // child's own map of C'_{l-1}.
        const int usz = a.hu * a.wu, csz = a.h * a.w;
        const int nparent = a.gxp * a.gyp;
        const __amdgpu_buffer_rsrc_t rsU = rsrc(u_cur, nparent * usz * 4), rsM = rsrc(code_cur, nparent * usz);
        const size_t cmap = (size_t)child_slot(g, a.l, c) * csz;
        const __amdgpu_buffer_rsrc_t rsC = rsrc(cp_prev + cmap, csz * 4);
        const __amdgpu_buffer_rsrc_t rsK = rsrc(code_prev + cmap, (BOTTOM || DMSTAR) ? csz : 0);
        // Element offset of each parent's map, or a large negative value for a
        // missing parent: with a lane's row offset added (also large negative
        // when the lane or row has no U_l entry), an entry exists exactly when
        // the sum is >= 0, so validity needs no lane masks per side.
        constexpr int kNone = -(1 << 30);
        int pbase[4];
#pragma unroll
        for (int side = 0; side < 4; ++side) {
            const int sx = (side & 2) ? 1 : -1, sy = (side & 1) ? 1 : -1;   // o_i of Eq. (5), i = side
            const int pb = parent_index(a.l, cb, sy), pa = parent_index(a.l, ca, sx);
            const bool ok = pb >= 0 && pb < a.gyp && pa >= 0 && pa < a.gxp && vxp[pa] && vyp[pb];
            pbase[side] = ok ? (pb * a.gxp + pa) * usz : kNone;
        }
        uint32_t (*ring)[kBtCols] = sR[wv];
        const int rx = C0 + t;                       // the lane's output column
        // While scattering, TILE = 60: lane t serves U_l column ux of the
        // sides 2p + h (h = t / 32) in the passes p = 0, 1 (output columns
        // [C0, C0 + 60) are reached only from columns C0/2 - 1 .. C0/2 + 30);
        // TILE = 64: lane t < 34 serves column ux of every side.
        constexpr int NP = TILE == 60 ? 2 : 4;       // passes (sides per lane)
        const int h = t >> 5;
        const int ux = (C0 >> 1) - 1 + (TILE == 60 ? (t & 31) : t);
        const bool lane_u = (TILE == 60 || t < TILE / 2 + 2) && ux >= 0 && ux < a.wu;
        const bool lane_o = t < TILE && rx < Cend;
        // Parent map offset of pass p for this lane; o_i of Eq. (5) along y
        // for the lane's sides (TILE = 60; along x it is fixed per pass).
        int pbl[NP];
        if constexpr (TILE == 60) {
            pbl[0] = h ? pbase[1] : pbase[0];
            pbl[1] = h ? pbase[3] : pbase[2];
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) pbl[p] = pbase[p];
        }
        const int sy_l = h ? 1 : -1;
        const int rp0 = (R0 - 1) >> 1, rp1 = ((R1 - 1) >> 1) + 1;

        struct UBuf { float u[NP]; int m[NP]; };
        struct OBuf { uint32_t vb[2]; float cv[2]; int cm[2]; };
        auto load_u = [&](int rp, UBuf& st) {
            const bool rok = lane_u && rp >= 0 && rp < a.hu;
            const int roff = rok ? rp * a.wu + ux : kNone;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int off = pbl[p] + roff;   // >= 0 exactly for an existing entry
                const bool ok = off >= 0;
                const float v =
                    __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsU, ok ? off * 4 : kOOB, 0, 0));
                st.m[p] = __builtin_amdgcn_raw_buffer_load_b8(rsM, ok ? off : kOOB, 0, 0);
                if constexpr (DMSTAR) st.m[p] &= 15;   // codes of a pooled level carry the entry mark above bit 3
                st.u[p] = ok ? v : -1.f;
            }
        };
        auto scatter = [&](int rp, const UBuf& st) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int sx = TILE == 60 ? (p ? 1 : -1) : ((p & 2) ? 1 : -1);   // side 2p + h, or p
                const int sy = TILE == 60 ? sy_l : ((p & 1) ? 1 : -1);
                const int ry = 2 * rp + code_my(st.m[p]) - 1 + sy, rxx = 2 * ux + code_mx(st.m[p]) - 1 + sx;
                // an entry (U = -inf: unreached; -1: no parent or column) whose target is in the tile
                const bool act = st.u[p] >= 0.f && (unsigned)(ry - R0) < (unsigned)(R1 - R0) &&
                                 (unsigned)(rxx - C0) < (unsigned)(Cend - C0);
                if (act) atomicMax(&ring[ry & (kBtRing - 1)][rxx - C0], enc(st.u[p]));
            }
        };
        auto collect = [&](int rp, OBuf& o) {
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const int ry = 2 * rp - 2 + dy;
                const bool rok = ry >= R0 && ry < R1;                          // uniform
                o.vb[dy] = (rok && lane_o) ? atomicExch(&ring[ry & (kBtRing - 1)][t], 0u) : 0u;
                // element offset in the child's map, used only where a tuple
                // arrived (DM*: at every cell, which may be an entry point)
                const int off = ry * a.w + rx;
                const bool need = DMSTAR ? (rok && lane_o) : o.vb[dy] != 0u;
                o.cv[dy] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsC, need ? off * 4 : kOOB, 0, 0));
                o.cm[dy] = __builtin_amdgcn_raw_buffer_load_b8(rsK, need ? off : kOOB, 0, 0);
            }
        };
        auto finish = [&](int rp, const OBuf& o) {
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const int ry = 2 * rp - 2 + dy;
                if (ry < R0 || ry >= R1 || !lane_o) continue;
                const uint32_t arrived = o.vb[dy];
                // DM*: an entry point where no tuple arrives starts one with its own value
                const bool ent = DMSTAR != 0 && (o.cm[dy] & kEntryBit);
                const uint32_t vb = ent && !arrived ? enc(0.f) : arrived;
                if constexpr (!BOTTOM) {
                    float uv;
                    if constexpr (DMSTAR == 2)   // start/end scores: the start value passes down unchanged
                        uv = arrived ? (ent ? fmaxf(dec(arrived), o.cv[dy]) : dec(arrived))
                                     : (ent ? o.cv[dy] : -INFINITY);
                    else
                        uv = vb ? o.cv[dy] + dec(vb) : -INFINITY;
                    u_prev[((size_t)c * a.h + ry) * a.w + rx] = uv;
                } else if (vb) {
                    const float uu = o.cv[dy] + dec(vb);
                    const int mm = DMSTAR ? (o.cm[dy] & 15) : o.cm[dy];
                    const int xy = 2 * ry + code_my(mm) - 1, xx = 2 * rx + code_mx(mm) - 1;
                    const unsigned long long hi = (unsigned long long)__float_as_uint(uu) << 32;
                    if constexpr (RECT) {
                        int qx, qy;
                        if (rect_target(g.rect, xx, xy, qx, qy)) {
                            const unsigned long long kb = hi | (0xFFFFFFFFull - (uint32_t)(qy * g.rect.W2o + qx));
                            mybest = kb > mybest ? kb : mybest;
                            atomicMax(&cell[(size_t)(qy >> 2) * g.rect.cw2 + (qx >> 2)],
                                      hi | (0xFFFFFFFFull - (uint32_t)(pidx * 16 + (qy & 3) * 4 + (qx & 3))));
                        }
                    } else {
                        const unsigned long long kb = hi | (0xFFFFFFFFull - (uint32_t)(xy * a.W2 + xx));
                        mybest = kb > mybest ? kb : mybest;
                        const unsigned long long kc =
                            hi | (0xFFFFFFFFull - (uint32_t)(c * 16 + (xy & 3) * 4 + (xx & 3)));
                        atomicMax(&sCell[((xy >> 2) - cyb) * NCX + ((xx >> 2) - cxb)], kc);
                    }
                }
            }
        };
        // Step rp: U_l row rp+1 is loading, row rp is scattered, output rows of
        // step rp are collected (their C' loads issued) and those of step rp-1
        // finished.  All loads are unconditional instructions, so no wait has
        // to drain the ones still in flight.
        UBuf u0, u1;
        OBuf o0, o1;
        o1.vb[0] = o1.vb[1] = 0u;
        o1.cv[0] = o1.cv[1] = 0.f;
        o1.cm[0] = o1.cm[1] = 0;
        load_u(rp0, u0);
        int rp = rp0;
        for (;;) {
            load_u(rp + 1, u1);
            scatter(rp, u0);
            wave_sync();
            collect(rp, o0);
            finish(rp - 1, o1);
            wave_sync();
            if (rp == rp1) {
                finish(rp, o0);
                break;
            }
            ++rp;
            load_u(rp + 1, u0);
            scatter(rp, u1);
            wave_sync();
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
    if constexpr (!BOTTOM) return;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)mybest, d), hi = __shfl_xor((uint32_t)(mybest >> 32), d);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        mybest = o > mybest ? o : mybest;
    }
    if (live && t == 0 && mybest) atomicMax(&best[scell], mybest);
    __syncthreads();
    for (int e = tid; e < ncy * NCX; e += 64 * kBtWaves) {
        const unsigned long long v = sCell[e];
        if (!v) continue;
        const int cy = cyb + e / NCX, cx = cxb + e % NCX;
        atomicMax(&cell[(size_t)cy * a.cw + cx], v);
    }
}

// A pyramid whose top is the bottom level: M' = every (p, q) of C_top.
template <bool RECT>
__device__ inline void top_reduce_body(const float* __restrict__ top, const Geom& g,
                                       unsigned long long* __restrict__ best, unsigned long long* __restrict__ cell,
                                       int bid) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.H2 * g.W2;
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i >= n) return;
    const int xx = i % g.W2, xy = (i / g.W2) % g.H2;
    const int c = i / ((size_t)g.W2 * g.H2);
    const unsigned long long hi = (unsigned long long)__float_as_uint(top[i]) << 32;
    if constexpr (RECT) {
        int qx, qy, px, py;
        if (!rect_target(g.rect, xx, xy, qx, qy)) return;
        rect_source(g.rect, c % g.gx[0], c / g.gx[0], px, py);
        atomicMax(&best[(py >> 2) * g.rect.cw1 + (px >> 2)], hi | (0xFFFFFFFFull - (uint32_t)(qy * g.rect.W2o + qx)));
        atomicMax(&cell[(size_t)(qy >> 2) * g.rect.cw2 + (qx >> 2)],
                  hi | (0xFFFFFFFFull - (uint32_t)((py * g.rect.W1o + px) * 16 + (qy & 3) * 4 + (qx & 3))));
        return;
    }
    atomicMax(&best[c], hi | (0xFFFFFFFFull - (uint32_t)(xy * g.W2 + xx)));
    atomicMax(&cell[(size_t)(xy >> 2) * ((g.W2 + 3) / 4) + (xx >> 2)],
              hi | (0xFFFFFFFFull - (uint32_t)(c * 16 + (xy & 3) * 4 + (xx & 3))));
}

// Reciprocal verification (Eq. (16)) and compaction in patch order (y1, x1).
__device__ inline void finalize_body(const unsigned long long* __restrict__ best,
                                     const unsigned long long* __restrict__ cell, const Geom& g,
                                     dm_match* __restrict__ out, int* __restrict__ n_out) {
    // kFinChunks passes of 1024 patches at a time: their BestAt keys are
    // loaded together, then the BestAt' entries they name, and only then are
    // the winners compacted pass by pass (two memory round trips per group
    // of passes instead of two per pass).
    constexpr int kFinChunks = 8;
    __shared__ int wsum[16];
    __shared__ int base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gx0 = g.gx[0], natom = g.gx[0] * g.gy[0], cw = (g.W2 + 3) / 4;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int start = 0; start < natom; start += 1024 * kFinChunks) {
        unsigned long long key[kFinChunks], cv[kFinChunks];
#pragma unroll
        for (int c = 0; c < kFinChunks; ++c) {
            const int j = start + c * 1024 + tid;
            key[c] = j < natom ? best[j] : 0ull;
        }
#pragma unroll
        for (int c = 0; c < kFinChunks; ++c) {
            cv[c] = 0ull;
            if (key[c]) {
                const uint32_t xi = 0xFFFFFFFFu - (uint32_t)key[c];
                const int xy = xi / g.W2, xx = xi % g.W2;
                cv[c] = cell[(size_t)(xy >> 2) * cw + (xx >> 2)];
            }
        }
#pragma unroll
        for (int c = 0; c < kFinChunks; ++c) {
            const int j = start + c * 1024 + tid;
            int flag = 0;
            dm_match m;
            if (key[c]) {
                const uint32_t xi = 0xFFFFFFFFu - (uint32_t)key[c];
                const int xy = xi / g.W2, xx = xi % g.W2;
                const unsigned long long expect = (key[c] & 0xFFFFFFFF00000000ull) |
                                                  (0xFFFFFFFFull - (uint32_t)(j * 16 + (xy & 3) * 4 + (xx & 3)));
                flag = cv[c] == expect;
                m.x1 = 2 + 4 * (j % gx0);
                m.y1 = 2 + 4 * (j / gx0);
                m.x2 = xx;
                m.y2 = xy;
                m.score = __uint_as_float((uint32_t)(key[c] >> 32));
            }
            const unsigned long long mask = __ballot(flag);
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            if (lane == 0) wsum[wave] = __popcll(mask);
            __syncthreads();
            int off = base;
            for (int w = 0; w < wave; ++w) off += wsum[w];
            if (flag) out[off + rank] = m;
            __syncthreads();
            if (tid == 0) {
                int tot = 0;
                for (int w = 0; w < 16; ++w) tot += wsum[w];
                base += tot;
            }
            __syncthreads();
        }
    }
    if (tid == 0) *n_out = base;
}

__device__ inline void fill_body(unsigned long long* p, size_t n, unsigned long long v, int bid) {
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Validity of each level's lattice along x and y (Eq. (7) with the boundary
// rule): level 0 is complete; an index exists above when one of its two
// children along that axis exists.  The grid of a level is the product of
// its two axes.
__device__ inline void valid_body(const Geom& g, uint8_t* __restrict__ vt) {
    __shared__ uint8_t cur[2][DM_MAX_DIM / 4 + 2], prv[2][DM_MAX_DIM / 4 + 2];
    for (int l = 0; l <= g.lmax; ++l) {
        for (int axis = 0; axis < 2; ++axis) {
            const int n = axis ? g.gy[l] : g.gx[l];
            const int np = l ? (axis ? g.gy[l - 1] : g.gx[l - 1]) : 0;
            for (int a = threadIdx.x; a < n; a += blockDim.x) {
                uint8_t v = 1;
                if (l) {
                    const int c0 = child_index(l, a, -1), c1 = child_index(l, a, 1);
                    v = (c0 >= 0 && c0 < np && prv[axis][c0]) || (c1 >= 0 && c1 < np && prv[axis][c1]);
                }
                cur[axis][a] = v;
                vt[(size_t)(2 * l + axis) * g.vstride + a] = v;
            }
        }
        __syncthreads();
        for (int axis = 0; axis < 2; ++axis) {
            const int n = axis ? g.gy[l] : g.gx[l];
            for (int a = threadIdx.x; a < n; a += blockDim.x) prv[axis][a] = cur[axis][a];
        }
        __syncthreads();
    }
}

template <bool RECT, int DMSTAR = 0>
__global__ __launch_bounds__(256) void k_backtrack(BtArgs a, const float* __restrict__ cp_prev,
                                                   const uint8_t* __restrict__ code_prev,
                                                   const float* __restrict__ u_cur,
                                                   const uint8_t* __restrict__ code_cur,
                                                   const float* __restrict__ top, const uint8_t* __restrict__ vt,
                                                   Geom g, float* __restrict__ u_prev,
                                                   unsigned long long* __restrict__ best,
                                                   unsigned long long* __restrict__ cell, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    bt_body<RECT, DMSTAR>(a, cp_prev, code_prev, u_cur, code_cur, top, vt, g, u_prev, best, cell, bid);
}

// DM* entry points: kEntryBit on the codes of the local maxima of C'_l (maps
// of existing patches only).  Block = (patch, band of kMarkRows rows, 256
// columns); a thread owns one column and walks down the band with the 3 x 3
// neighbourhood in registers.  It loads one value per row, kMarkAhead rows
// at a time (the walk is bound by load latency, not by bytes), and sets
// the bit with a store that nothing waits for; the left and right values
// come from the neighbouring lanes, and the first and last lanes of a wave
// load the column beside the wave.  The code array is 256-byte aligned in
// the workspace, so the word around any of its bytes lies inside it.  Neighbours outside the
// map are -inf, which every comparison passes: the same decision as
// local_max, which skips them.
constexpr int kMarkRows = 32;
constexpr int kMarkAhead = 8;
static_assert(kMarkRows % kMarkAhead == 0, "bands are whole groups of rows");
__global__ __launch_bounds__(256) void k_mark_entries(const float* __restrict__ cp, uint8_t* __restrict__ code,
                                                      const uint8_t* __restrict__ vt, Geom g, int l, int nxt,
                                                      int nband) {
    const int h = g.h[l + 1], w = g.w[l + 1];
    const int bid = blockIdx.x;
    const int xt = bid % nxt, rest = bid / nxt, band = rest % nband, c = rest / nband;   // uniform
    const int cb = c / g.gx[l], ca = c - cb * g.gx[l];
    if (!vtab(vt, g, l, 0)[ca] || !vtab(vt, g, l, 1)[cb]) return;
    const int lane = (int)threadIdx.x & 63;
    const int x = xt * 256 + (int)threadIdx.x;
    if (__builtin_amdgcn_readfirstlane(xt * 256 + ((int)threadIdx.x & ~63)) >= w) return;   // whole wave past the map
    const bool in = x < w;
    // the column this lane loads besides its own: left of the wave (lane 0) or right of it (lane 63)
    const int xh = lane == 0 ? x - 1 : x + 1;
    const bool hok = (lane == 0 || lane == 63) && xh >= 0 && xh < w;
    const size_t pm = (size_t)h * w;
    const float* __restrict__ m = cp + (size_t)c * pm;
    uint8_t* __restrict__ k = code + (size_t)c * pm;
    const int y0 = band * kMarkRows, y1 = min(y0 + kMarkRows, h);
    auto centre = [&](int y) { return (in && y >= 0 && y < h) ? m[(size_t)y * w + x] : -INFINITY; };
    auto side = [&](int y) { return (hok && y >= 0 && y < h) ? m[(size_t)y * w + xh] : -INFINITY; };
    // left and right values of a row from the lanes beside (the wave's edge lanes: their own side value)
    auto spread = [&](float vc, float vh, float& vl, float& vr) {
        const float up = __shfl_up(vc, 1), dn = __shfl_down(vc, 1);
        vl = lane == 0 ? vh : up;
        vr = lane == 63 ? vh : dn;
    };
    float ul, uc, ur, ml, mc, mr;
    uc = centre(y0 - 1);
    spread(uc, side(y0 - 1), ul, ur);
    mc = centre(y0);
    spread(mc, side(y0), ml, mr);
    for (int yb = y0; yb < y1; yb += kMarkAhead) {
        float cn[kMarkAhead], hn[kMarkAhead];   // rows yb + 1 .. yb + kMarkAhead, loaded together
#pragma unroll
        for (int i = 0; i < kMarkAhead; ++i) {
            cn[i] = centre(yb + 1 + i);
            hn[i] = side(yb + 1 + i);
        }
#pragma unroll
        for (int i = 0; i < kMarkAhead; ++i) {
            const int y = yb + i;
            float dl, dr;
            const float dc = cn[i];
            spread(dc, hn[i], dl, dr);
            const float v = mc;
            // before it in raster order: strictly above; after it: not below
            const bool e = v > 0.f && v > ul && v > uc && v > ur && v > ml && v >= mr && v >= dl && v >= dc && v >= dr;
            if (in && y < y1 && e) {
                // no-return atomic OR on the aligned word holding the byte: the walk does
                // not wait for a load of the code (the other bytes stay as they are)
                const uintptr_t ad = reinterpret_cast<uintptr_t>(k + (size_t)y * w + x);
                atomicOr(reinterpret_cast<unsigned int*>(ad & ~uintptr_t(3)), (unsigned int)kEntryBit << (8 * (ad & 3)));
            }
            ul = ml, uc = mc, ur = mr;
            ml = dl, mc = dc, mr = dr;
        }
    }
}

template <bool RECT, int TILE, bool BOTTOM, int DMSTAR = 0>
__global__ __launch_bounds__(64 * kBtWaves) void k_backtrack_stream(
    BtStreamArgs a, const float* __restrict__ cp_prev, const uint8_t* __restrict__ code_prev,
    const float* __restrict__ u_cur, const uint8_t* __restrict__ code_cur, const uint8_t* __restrict__ vt, Geom g,
    float* __restrict__ u_prev, unsigned long long* __restrict__ best, unsigned long long* __restrict__ cell,
    int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    bt_stream_body<RECT, TILE, BOTTOM, DMSTAR>(a, cp_prev, code_prev, u_cur, code_cur, vt, g, u_prev, best, cell,
                                               bid);
}

template <bool RECT>
__global__ void k_top_reduce(const float* __restrict__ top, Geom g, unsigned long long* __restrict__ best,
                             unsigned long long* __restrict__ cell) {
    top_reduce_body<RECT>(top, g, best, cell, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_finalize(const unsigned long long* __restrict__ best,
                                                   const unsigned long long* __restrict__ cell, Geom g,
                                                   dm_match* __restrict__ out, int* __restrict__ n_out) {
    finalize_body(best, cell, g, out, n_out);
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) { fill_body(p, n, v, blockIdx.x); }

__global__ __launch_bounds__(1024) void k_valid_init(Geom g, uint8_t* __restrict__ vt) { valid_body(g, vt); }

struct BtJob {
    BtArgs a;
    const float* cp_prev;
    const uint8_t* code_prev;
    const float* u_cur;
    const uint8_t* code_cur;
    const float* top;
    const uint8_t* vt;
    Geom g;
    float* u_prev;
    unsigned long long *best, *cell;
    static __device__ void run(const BtJob& j, int v) {
        bt_body<false>(j.a, j.cp_prev, j.code_prev, j.u_cur, j.code_cur, j.top, j.vt, j.g, j.u_prev, j.best, j.cell,
                       v);
    }
};

template <int TILE, bool BOTTOM>
struct BtStreamJob {
    BtStreamArgs a;
    const float* cp_prev;
    const uint8_t* code_prev;
    const float* u_cur;
    const uint8_t* code_cur;
    const uint8_t* vt;
    Geom g;
    float* u_prev;
    unsigned long long *best, *cell;
    static __device__ void run(const BtStreamJob& j, int v) {
        bt_stream_body<false, TILE, BOTTOM>(j.a, j.cp_prev, j.code_prev, j.u_cur, j.code_cur, j.vt, j.g, j.u_prev,
                                            j.best, j.cell, v);
    }
};

struct TopReduceJob {
    const float* top;
    Geom g;
    unsigned long long *best, *cell;
    static __device__ void run(const TopReduceJob& j, int v) { top_reduce_body<false>(j.top, j.g, j.best, j.cell, v); }
};

struct FinalizeJob {
    const unsigned long long *best, *cell;
    Geom g;
    dm_match* out;
    int* n_out;
    static __device__ void run(const FinalizeJob& j, int) { finalize_body(j.best, j.cell, j.g, j.out, j.n_out); }
};

struct FillJob {
    unsigned long long* p;
    size_t n;
    unsigned long long v;
    static __device__ void run(const FillJob& j, int v) { fill_body(j.p, j.n, j.v, v); }
};

struct ValidJob {
    Geom g;
    uint8_t* vt;
    static __device__ void run(const ValidJob& j, int) { valid_body(j.g, j.vt); }
};

// Tiled form of backtracking step l (reads level l, produces level l-1).
BtArgs make_bt_args(int l, const Geom& g, int& nblocks, size_t& smem) {
    BtArgs a;
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
    a.is_bottom = (l == 1);
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
    a.W2 = g.W2;
    a.cw = (g.W2 + 3) / 4;
    a.ncy = a.TR / 2 + 2;
    a.ncx = a.TC / 2 + 2;
    a.cy0 = a.cx0 = 0;
    smem = (size_t)4 * a.CB * a.TR * a.TC * sizeof(uint32_t) + ((size_t)a.CB + (size_t)a.ncy * a.ncx) * 8 +
           (size_t)5 * a.CB * sizeof(int);
    nblocks = a.n_cblk * a.n_rt * n_ct;
    a.f_t = make_fastdiv(a.TR * a.TC);
    a.f_tc = make_fastdiv(a.TC);
    a.f_nr = make_fastdiv((a.TR / 2 + 2) * (a.TC / 2 + 2));
    a.f_rwd = make_fastdiv(a.TC / 2 + 2);
    return a;
}

// The streaming form serves every step below the top whose child maps are at
// least 32 columns wide and whose parent arrays (U_l) stay below 2^31 bytes
// (buffer offsets; a child's map has a descriptor of its own).
bool use_bt_stream(int l, const Geom& g) {
    if (l == g.lmax || g.w[l] < 32) return false;
    return (double)g.gx[l] * g.gy[l] * g.h[l + 1] * g.w[l + 1] * 4 < 2.0e9;
}

// Output columns per wave for child maps w wide: the form with the shorter
// time per row of the map (a 60-column wave takes about 0.76 of a 64-column
// wave's time, measured at 512x256, but more waves are needed when
// ceil(w / 60) > ceil(w / 64)).
int bt_tile(int w) {
    const int n60 = (w + 59) / 60, n64 = (w + 63) / 64;
    return n60 * 76 <= n64 * 100 ? 60 : 64;
}

// Streaming form with bands of tr rows (even, at most kBtMaxTR).
BtStreamArgs make_bt_stream_args(int l, const Geom& g, int tr, int& nblocks) {
    BtStreamArgs b;
    b.l = l;
    b.gxp = g.gx[l];
    b.gyp = g.gy[l];
    b.gxc = g.gx[l - 1];
    b.gyc = g.gy[l - 1];
    b.h = g.h[l];
    b.w = g.w[l];
    b.hu = g.h[l + 1];
    b.wu = g.w[l + 1];
    b.is_bottom = (l == 1);
    tr = tr < 2 ? 2 : (tr > kBtMaxTR ? kBtMaxTR : tr & ~1);
    b.TR = b.h < tr ? ((b.h + 1) & ~1) : tr;
    b.n_band = (b.h + b.TR - 1) / b.TR;
    b.tile = bt_tile(b.w);
    b.n_ct = (b.w + b.tile - 1) / b.tile;
    b.n_cgrp = (b.gxc * b.gyc + kBtWaves - 1) / kBtWaves;
    b.W2 = g.W2;
    b.cw = (g.W2 + 3) / 4;
    nblocks = b.n_cgrp * b.n_ct * b.n_band;
    return b;
}

}  // namespace

template <>
hipError_t launch_backtrack<float>(int l, const float* cp_prev, const uint8_t* code_prev, const float* u_cur,
                                   const uint8_t* code_cur, const float* top, const uint8_t* vt, const Geom& g,
                                   float* u_prev, uint64_t* best, uint64_t* cell, hipStream_t s) {
    if (use_bt_stream(l, g) && !(g.dmstar && g.rect.on)) {
        int nb;
        const BtStreamArgs b = make_bt_stream_args(l, g, kBtTR, nb);
        auto* b64 = (unsigned long long*)best;
        auto* c64 = (unsigned long long*)cell;
        const dim3 grid(((nb + 7) / 8) * 8), block(64 * kBtWaves);
#define DM_BT_STREAM(R, T, B, D)                                                                                    \
    hipLaunchKernelGGL((k_backtrack_stream<R, T, B, D>), grid, block, 0, s, b, cp_prev, code_prev, u_cur, code_cur, \
                       vt, g, u_prev, b64, c64, nb)
        // The rectified (invariant) form differs from the plain one at the
        // bottom level only; so do DM*'s two scoring schemes, the other way round.
        if (g.dmstar) {
            if (b.is_bottom && b.tile == 60) DM_BT_STREAM(false, 60, true, 1);
            else if (b.is_bottom) DM_BT_STREAM(false, 64, true, 1);
            else if (g.dmstar == 2 && b.tile == 60) DM_BT_STREAM(false, 60, false, 2);
            else if (g.dmstar == 2) DM_BT_STREAM(false, 64, false, 2);
            else if (b.tile == 60) DM_BT_STREAM(false, 60, false, 1);
            else DM_BT_STREAM(false, 64, false, 1);
        } else if (b.is_bottom) {
            if (g.rect.on && b.tile == 60) DM_BT_STREAM(true, 60, true, 0);
            else if (g.rect.on) DM_BT_STREAM(true, 64, true, 0);
            else if (b.tile == 60) DM_BT_STREAM(false, 60, true, 0);
            else DM_BT_STREAM(false, 64, true, 0);
        } else {
            if (b.tile == 60) DM_BT_STREAM(false, 60, false, 0);
            else DM_BT_STREAM(false, 64, false, 0);
        }
#undef DM_BT_STREAM
        return hipGetLastError();
    }
    int nblocks;
    size_t smem;
    const BtArgs a = make_bt_args(l, g, nblocks, smem);
    const dim3 grid(((nblocks + 7) / 8) * 8);
    if (g.dmstar == 2)
        hipLaunchKernelGGL((k_backtrack<false, 2>), grid, dim3(256), smem, s, a, cp_prev, code_prev, u_cur,
                           code_cur, top, vt, g, u_prev, (unsigned long long*)best, (unsigned long long*)cell, nblocks);
    else if (g.dmstar)
        hipLaunchKernelGGL((k_backtrack<false, 1>), grid, dim3(256), smem, s, a, cp_prev, code_prev, u_cur,
                           code_cur, top, vt, g, u_prev, (unsigned long long*)best, (unsigned long long*)cell, nblocks);
    else if (g.rect.on)
        hipLaunchKernelGGL(k_backtrack<true>, grid, dim3(256), smem, s, a, cp_prev, code_prev, u_cur, code_cur, top,
                           vt, g, u_prev, (unsigned long long*)best, (unsigned long long*)cell, nblocks);
    else
        hipLaunchKernelGGL(k_backtrack<false>, grid, dim3(256), smem, s, a, cp_prev, code_prev, u_cur, code_cur, top,
                           vt, g, u_prev, (unsigned long long*)best, (unsigned long long*)cell, nblocks);
    return hipGetLastError();
}

JobRec bt_job(int l, const float* cp_prev, const uint8_t* code_prev, const float* u_cur, const uint8_t* code_cur,
              const float* top, const uint8_t* vt, const Geom& g, float* u_prev, uint64_t* best, uint64_t* cell,
              int tr) {
    JobRec r;
    auto* b64 = (unsigned long long*)best;
    auto* c64 = (unsigned long long*)cell;
    if (use_bt_stream(l, g)) {
        int nb;
        const BtStreamArgs b = make_bt_stream_args(l, g, tr, nb);
        if (b.tile == 60 && b.is_bottom)
            r.set(JK_BT_STREAM_BOT, nb, 0,
                  BtStreamJob<60, true>{b, cp_prev, code_prev, u_cur, code_cur, vt, g, u_prev, b64, c64});
        else if (b.tile == 60)
            r.set(JK_BT_STREAM, nb, 0,
                  BtStreamJob<60, false>{b, cp_prev, code_prev, u_cur, code_cur, vt, g, u_prev, b64, c64});
        else if (b.is_bottom)
            r.set(JK_BT_STREAM64_BOT, nb, 0,
                  BtStreamJob<64, true>{b, cp_prev, code_prev, u_cur, code_cur, vt, g, u_prev, b64, c64});
        else
            r.set(JK_BT_STREAM64, nb, 0,
                  BtStreamJob<64, false>{b, cp_prev, code_prev, u_cur, code_cur, vt, g, u_prev, b64, c64});
        return r;
    }
    int nb;
    size_t smem;
    const BtArgs a = make_bt_args(l, g, nb, smem);
    r.set(JK_BT, nb, smem, BtJob{a, cp_prev, code_prev, u_cur, code_cur, top, vt, g, u_prev, b64, c64});
    return r;
}

JobRec top_reduce_job(const float* top, const Geom& g, uint64_t* best, uint64_t* cell) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.H2 * g.W2;
    JobRec r;
    r.set(JK_TOP_REDUCE, (int)((n + 255) / 256), 0,
          TopReduceJob{top, g, (unsigned long long*)best, (unsigned long long*)cell});
    return r;
}

JobRec finalize_job(const uint64_t* best, const uint64_t* cell, const Geom& g, dm_match* out, int* n_out) {
    JobRec r;
    r.set(JK_FINALIZE, 1, 0, FinalizeJob{(const unsigned long long*)best, (const unsigned long long*)cell, g, out, n_out});
    return r;
}

JobRec fill_job(uint64_t* p, size_t n, uint64_t v) {
    JobRec r;
    r.set(JK_FILL, (int)((n + 255) / 256), 0, FillJob{(unsigned long long*)p, n, (unsigned long long)v});
    return r;
}

JobRec valid_job(const Geom& g, uint8_t* vt) {
    JobRec r;
    r.set(JK_VALID, 1, 0, ValidJob{g, vt});
    return r;
}

hipError_t launch_group_bt(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_BT: return launch_grouped<BtJob, 256, 1>(gl, s);
        case JK_BT_STREAM: return launch_grouped<BtStreamJob<60, false>, 64 * kBtWaves, 1>(gl, s);
        case JK_BT_STREAM64: return launch_grouped<BtStreamJob<64, false>, 64 * kBtWaves, 1>(gl, s);
        case JK_BT_STREAM_BOT: return launch_grouped<BtStreamJob<60, true>, 64 * kBtWaves, 1>(gl, s);
        case JK_BT_STREAM64_BOT: return launch_grouped<BtStreamJob<64, true>, 64 * kBtWaves, 1>(gl, s);
        case JK_TOP_REDUCE: return launch_grouped<TopReduceJob, 256, 1>(gl, s);
        case JK_FINALIZE: return launch_grouped<FinalizeJob, 1024, 1>(gl, s);
        case JK_FILL: return launch_grouped<FillJob, 256, 1>(gl, s);
        case JK_VALID: return launch_grouped<ValidJob, 1024, 1>(gl, s);
        default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_top_reduce<float>(const float* top, const Geom& g, uint64_t* best, uint64_t* cell,
                                    hipStream_t s) {
    const size_t n = (size_t)g.gx[0] * g.gy[0] * g.H2 * g.W2;
    if (g.rect.on)
        hipLaunchKernelGGL(k_top_reduce<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, top, g,
                           (unsigned long long*)best, (unsigned long long*)cell);
    else
        hipLaunchKernelGGL(k_top_reduce<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, top, g,
                           (unsigned long long*)best, (unsigned long long*)cell);
    return hipGetLastError();
}

hipError_t launch_finalize(const uint64_t* best, const uint64_t* cell, const Geom& g, dm_match* out, int* n_out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, (const unsigned long long*)best,
                       (const unsigned long long*)cell, g, out, n_out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (unsigned long long*)p, n,
                       (unsigned long long)v);
    return hipGetLastError();
}

hipError_t launch_mark_entries(int l, const float* cp, uint8_t* code, const uint8_t* vt, const Geom& g,
                               hipStream_t s) {
    const int h = g.h[l + 1], w = g.w[l + 1], np = g.gx[l] * g.gy[l];
    if (!h || !w || !np) return hipSuccess;
    const int nxt = (w + 255) / 256, nband = (h + kMarkRows - 1) / kMarkRows;
    const long long nb = (long long)np * nband * nxt;
    if (nb >= (1ll << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mark_entries, dim3((unsigned)nb), dim3(256), 0, s, cp, code, vt, g, l, nxt, nband);
    return hipGetLastError();
}

hipError_t launch_valid_init(const Geom& g, uint8_t* vt, hipStream_t s) {
    hipLaunchKernelGGL(k_valid_init, dim3(1), dim3(1024), 0, s, g, vt);
    return hipGetLastError();
}

}  // namespace dm
