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
#include <type_traits>

#include "dm_group.h"

namespace dm {
namespace {

struct LevelArgs {
    int l;
    int gx, gy, gxc, gyc;  // lattices of this level and of the children's
    int h, w, hp, wp;      // maps of this level (C_l) and pooled (C'_l)
    int TRo, TCo, PB;      // tile: pooled rows, pooled cols, parents per block
    int n_pblk, n_rt;      // block grid factors
    FastDiv f_ra, f_rw, f_tile, f_tco;  // divisions by RA, RW, TRo*TCo, TCo (element indices < 2^13)
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

// Blocks are dealt to the 8 XCDs round-robin by index; renumber them so that
// each XCD works through a contiguous range of the logical order (parent
// fastest), keeping parents that share children on one L2.
__device__ inline int xcd_block(int nblocks) {
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Per-parent data of a block, computed once: the child maps (null if the
// child does not exist) and 1/|V|.
template <typename T>
struct ParentLDS {
    const T* cmap[4];
    T inv;
    int valid;
};

template <typename T>
__device__ inline void load_parents(const LevelArgs& a, const Geom& g, int pbase, const uint8_t* vxp,
                                    const uint8_t* vyp, const uint8_t* vxc, const uint8_t* vyc, const T* prev,
                                    ParentLDS<T>* sp) {
    const size_t hw = (size_t)a.h * a.w;
    for (int k = threadIdx.x; k < a.PB; k += blockDim.x) {
        const Parent<T> pi = parent_info<T>(a, pbase + k, vxp, vyp, vxc, vyc);
        ParentLDS<T> r;
#pragma unroll
        for (int ky = 0; ky < 2; ++ky)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx)
                r.cmap[2 * ky + kx] =
                    (pi.cb[ky] >= 0 && pi.ca[kx] >= 0)
                        ? prev + (size_t)child_slot(g, a.l, pi.cb[ky] * a.gxc + pi.ca[kx]) * hw
                        : nullptr;
        r.inv = pi.inv;
        r.valid = pi.valid;
        sp[k] = r;
    }
}

// max(A_l(P, q), 0) from the staged parent data, or -1 off the map / parent.
template <typename T>
__device__ inline T staged_aggregate(const LevelArgs& a, const ParentLDS<T>& pr, const T* __restrict__ prev, int qy,
                                     int qx) {
    if (!pr.valid || qy < 0 || qy >= a.h || qx < 0 || qx >= a.w) return T(-1);
    T acc = 0;
#pragma unroll
    for (int ky = 0; ky < 2; ++ky) {
        const int y = qy + 2 * ky - 1;
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
            const int x = qx + 2 * kx - 1;
            const T* m = pr.cmap[2 * ky + kx];
            if (m && y >= 0 && y < a.h && x >= 0 && x < a.w) acc += m[y * a.w + x];
        }
    }
    acc *= pr.inv;
    return acc > T(0) ? acc : T(0);
}

template <typename T>
__device__ inline void level_pool_body(const LevelArgs& a, const T* __restrict__ prev, const uint8_t* __restrict__ vt,
                                       const Geom& g, T lam, T* __restrict__ cp, uint8_t* __restrict__ code, int bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ParentLDS<T>* sp = (ParentLDS<T>*)smem_raw;
    T* sA = (T*)(smem_raw + ((a.PB * sizeof(ParentLDS<T>) + 15) & ~size_t(15)));
    const int rest = bid / a.n_pblk, pblk = bid - rest * a.n_pblk;   // once per block (scalar)
    const int ct = rest / a.n_rt, R0 = (rest - ct * a.n_rt) * a.TRo, C0 = ct * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    load_parents<T>(a, g, pblk * a.PB, vxp, vyp, vxc, vyc, prev, sp);
    __syncthreads();
    const int RW = 2 * a.TCo + 1, RA = (2 * a.TRo + 1) * RW, total = a.PB * RA;
    // Phase 1: stage max(A, 0) on the pooling footprint; 4 elements per
    // thread and pass so that their child loads are in flight together.
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * 256) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * 256;
            v[u] = T(-1);
            if (e < total) {
                const int k = fdiv(e, a.f_ra), rem = e - k * RA;
                const int ry = fdiv(rem, a.f_rw);
                v[u] = staged_aggregate(a, sp[k], prev, 2 * R0 - 1 + ry, 2 * C0 - 1 + rem - ry * RW);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * 256 < total) sA[e0 + u * 256] = v[u];
    }
    __syncthreads();
    // Phase 2: 3x3 / stride-2 max-pool, first maximum in code order, rectify.
    for (int e = threadIdx.x; e < a.PB * a.TRo * a.TCo; e += 256) {
        const int k = fdiv(e, a.f_tile), rem = e - k * (a.TRo * a.TCo);
        const int orow = fdiv(rem, a.f_tco), ocol = rem - orow * a.TCo;
        const int P = pblk * a.PB + k, r = R0 + orow, c = C0 + ocol;
        if (!sp[k].valid || r >= a.hp || c >= a.wp) continue;
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

// Row-streaming form of k_level_pool for maps at least 32 pooled columns
// wide.  One wave owns a parent, a band of pooled rows and up to 128 pooled
// columns, and walks down the rows of A.  Lane t owns the 4 A columns
// X0 + 4t .. X0 + 4t + 3 (X0 = 2 C0 - 1) and the pooled columns C0 + 2t,
// C0 + 2t + 1; the fifth A value the second window needs comes from lane
// t + 1 (lane 63: a halo column every lane loads).  Each A row is computed
// once from 4 child rows (no branches around the loads: clamped addresses,
// then selects), pooled horizontally in registers and merged into a running
// vertical maximum; the loads of the next row are in flight meanwhile.
// Scanning my outer and mx inner with strict comparisons keeps the first
// maximum in code order, as the direct 3x3 scan does.
constexpr int kStreamCols = 128;     // pooled columns per wave
constexpr int kOOB = 0x7ffffff0;     // buffer byte offset past any row
constexpr int kStreamWaves = 4;      // independent waves per block

struct StreamArgs {
    int l;
    int gx, gy, gxc, gyc;
    int h, w, hp, wp;
    int TRo, n_band, n_ct, n_items;
    int vec;                         // 2: w % 4 == 0, 16-byte child row pieces; 1: w even, 8-byte pieces; 0: odd w
    int narrow;                      // pooled maps <= 64 wide (and vec): several bands per wave
    int lgl;                         // narrow: log2 of the lanes per band (the wave walks 64 >> lgl bands)
};

// Child values of one A row for a lane: v[k][j] for its 4 columns, hv[k] for
// the halo column (0 where the child, its row or the column does not exist).
struct RowBuf {
    float v[4][4];
    float hv[4];
};

// Vector elements are read with __uint_as_float(f[j]): a bit cast applied to
// an element expression of an ext_vector reads element 0 on this compiler.
// Buffer descriptor of one child row: loads at byte offsets outside
// [0, nbytes) return 0 in hardware, which is exactly the rule for child
// values outside the map (and nbytes = 0 for a missing child or row).
__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const float* row, int nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), (short)0, nbytes, 0x00020000);
}

template <int VEC>
__device__ inline void load_row(const StreamArgs& a, const float* prev, const float* const cmap[4], int y, int X0,
                                int t, RowBuf& b) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int yy = y + 2 * (k >> 1) - 1, dx = 2 * (k & 1) - 1;
        const bool rok = cmap[k] != nullptr && yy >= 0 && yy < a.h;     // uniform over the wave
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(rok ? cmap[k] + (size_t)yy * a.w : prev, rok ? a.w * 4 : 0);
        // Column offsets are never negative: a column left of the row gets
        // kOOB (a byte offset past any row), so that each load is in or out of
        // range on its own whatever the compiler folds into immediate offsets.
        const int s0 = X0 + 4 * t + dx;   // >= -2
        if ((k & 1) && VEC == 2) {   // s0 = 2 C0 + 4t >= 0: 16-byte aligned, entirely inside or outside the row
            const auto f = __builtin_amdgcn_raw_buffer_load_b128(rs, s0 * 4, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) b.v[k][j] = __uint_as_float(f[j]);
        } else {       // s0 = 2 C0 + 4t - 2 or 2 C0 + 4t (w even): two 8-byte halves, each inside or outside
            const auto f0 = __builtin_amdgcn_raw_buffer_load_b64(rs, s0 >= 0 ? s0 * 4 : kOOB, 0, 0);
            const auto f1 = __builtin_amdgcn_raw_buffer_load_b64(rs, s0 * 4 + 8, 0, 0);
            b.v[k][0] = __uint_as_float(f0[0]);
            b.v[k][1] = __uint_as_float(f0[1]);
            b.v[k][2] = __uint_as_float(f1[0]);
            b.v[k][3] = __uint_as_float(f1[1]);
        }
        b.hv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (X0 + 4 * 64 + dx) * 4, 0, 0));
    }
}

// Horizontal first maxima (value, mx code 0..2) of the lane's two windows.
__device__ inline void pool_row(const StreamArgs& a, const RowBuf& b, float inv, int y, int X0, int t, float hv[2],
                                int hk[2]) {
    const bool yin = y >= 0 && y < a.h;
    float av[5];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float s = (((0.f + b.v[0][j]) + b.v[1][j]) + b.v[2][j]) + b.v[3][j];
        const float m = s * inv;
        const int x = X0 + 4 * t + j;
        av[j] = (yin && x >= 0 && x < a.w) ? fmaxf(m, 0.f) : -1.f;
    }
    {
        const float s = (((0.f + b.hv[0]) + b.hv[1]) + b.hv[2]) + b.hv[3];
        const float m = s * inv;
        const float halo = (yin && X0 + 4 * 64 < a.w) ? fmaxf(m, 0.f) : -1.f;
        const float nb = __shfl_down(av[0], 1);
        av[4] = t == 63 ? halo : nb;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const float v0 = av[2 * q], v1 = av[2 * q + 1], v2 = av[2 * q + 2];
        float best = v0;
        int k = 0;
        if (v1 > best) { best = v1; k = 1; }
        if (v2 > best) { best = v2; k = 2; }
        hv[q] = best;
        hk[q] = k;
    }
}

// Narrow maps (at most 64 pooled columns, w even): the wave splits into
// groups of L = 2^lgl lanes (L >= half the pooled width), each walking its
// own band of the same parent, lane tt = t % L owning the A columns
// 4 tt - 1 .. 4 tt + 3.  Rows differ between the groups, so each child has a
// descriptor over its whole map and a lane's offset is kOOB wherever its row
// or columns fall outside (an even w keeps every 8-byte piece, and w % 4 ==
// 0 every 16-byte piece, wholly inside or outside a row).  Same sums, same
// comparisons: the values equal those of the 64-lane form.
template <int VEC>
__device__ inline void load_row_narrow(const StreamArgs& a, const __amdgpu_buffer_rsrc_t rs[4], const bool ex[4],
                                       int y, int tt, int L, RowBuf& b) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int yy = y + 2 * (k >> 1) - 1, dx = 2 * (k & 1) - 1;
        const bool rok = ex[k] && yy >= 0 && yy < a.h;
        const int rowb = yy * a.w;
        const int s0 = 4 * tt - 1 + dx;   // -2 .. 125
        if ((k & 1) && VEC == 2) {   // s0 = 4 tt: 16 bytes inside or outside the row
            const auto f = __builtin_amdgcn_raw_buffer_load_b128(rs[k], rok && s0 < a.w ? (rowb + s0) * 4 : kOOB, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) b.v[k][j] = __uint_as_float(f[j]);
        } else {       // s0 = 4 tt - 2 or 4 tt (w even): two 8-byte halves
            const auto f0 = __builtin_amdgcn_raw_buffer_load_b64(
                rs[k], rok && s0 >= 0 && s0 < a.w ? (rowb + s0) * 4 : kOOB, 0, 0);
            const auto f1 =
                __builtin_amdgcn_raw_buffer_load_b64(rs[k], rok && s0 + 2 < a.w ? (rowb + s0 + 2) * 4 : kOOB, 0, 0);
            b.v[k][0] = __uint_as_float(f0[0]);
            b.v[k][1] = __uint_as_float(f0[1]);
            b.v[k][2] = __uint_as_float(f1[0]);
            b.v[k][3] = __uint_as_float(f1[1]);
        }
        const int hx = 4 * L - 1 + dx;   // the halo column of the group
        b.hv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs[k], rok && hx < a.w ? (rowb + hx) * 4 : kOOB,
                                                                        0, 0));
    }
}

__device__ inline void pool_row_narrow(const StreamArgs& a, const RowBuf& b, float inv, int y, int tt, int L,
                                       float hv[2], int hk[2]) {
    const bool yin = y >= 0 && y < a.h;
    float av[5];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float s = (((0.f + b.v[0][j]) + b.v[1][j]) + b.v[2][j]) + b.v[3][j];
        const float m = s * inv;
        const int x = 4 * tt - 1 + j;
        av[j] = (yin && x >= 0 && x < a.w) ? fmaxf(m, 0.f) : -1.f;
    }
    {
        const float s = (((0.f + b.hv[0]) + b.hv[1]) + b.hv[2]) + b.hv[3];
        const float m = s * inv;
        const float halo = (yin && 4 * L - 1 < a.w) ? fmaxf(m, 0.f) : -1.f;
        const float nb = __shfl_down(av[0], 1);
        av[4] = tt == L - 1 ? halo : nb;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const float v0 = av[2 * q], v1 = av[2 * q + 1], v2 = av[2 * q + 2];
        float best = v0;
        int k = 0;
        if (v1 > best) { best = v1; k = 1; }
        if (v2 > best) { best = v2; k = 2; }
        hv[q] = best;
        hk[q] = k;
    }
}

template <int VEC>
__device__ inline void level_narrow_body(const StreamArgs& a, const float* __restrict__ prev, const float* const cmap[4],
                                         float inv, int P, int band2, int t, float lam, float* __restrict__ cp,
                                         uint8_t* __restrict__ code) {
    const int L = 1 << a.lgl, tt = t & (L - 1), hh = t >> a.lgl;
    const int R0 = ((64 >> a.lgl) * band2 + hh) * a.TRo, R1 = min(R0 + a.TRo, a.hp);   // this group's band (may be empty)
    __amdgpu_buffer_rsrc_t rs[4];
    bool ex[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ex[k] = cmap[k] != nullptr;
        rs[k] = row_rsrc(ex[k] ? cmap[k] : prev, ex[k] ? a.h * a.w * 4 : 0);
    }
    RowBuf b0, b1;
    float pv[2], hv[2];
    int pk[2], hk[2];
    load_row_narrow<VEC>(a, rs, ex, 2 * R0 - 1, tt, L, b0);
    load_row_narrow<VEC>(a, rs, ex, 2 * R0, tt, L, b1);
    pool_row_narrow(a, b0, inv, 2 * R0 - 1, tt, L, pv, pk);
    for (int i = 0; i < a.TRo; ++i) {   // the same count in every group
        const int r = R0 + i;
        load_row_narrow<VEC>(a, rs, ex, 2 * r + 1, tt, L, b0);
        float best[2];
        int bk[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) { best[q] = pv[q]; bk[q] = pk[q]; }
        pool_row_narrow(a, b1, inv, 2 * r, tt, L, hv, hk);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (hv[q] > best[q]) { best[q] = hv[q]; bk[q] = 3 + hk[q]; }
        load_row_narrow<VEC>(a, rs, ex, 2 * r + 2, tt, L, b1);
        pool_row_narrow(a, b0, inv, 2 * r + 1, tt, L, pv, pk);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (pv[q] > best[q]) { best[q] = pv[q]; bk[q] = 6 + pk[q]; }
            const int u = 2 * tt + q;
            if (r < R1 && u < a.wp) {
                const size_t o = ((size_t)P * a.hp + r) * a.wp + u;
                cp[o] = rect_pow(best[q], lam);
                code[o] = (uint8_t)bk[q];
            }
        }
    }
}

// Maps whose width is not a multiple of 4 (rows not 16-byte aligned): lane t
// holds the A columns X0 + 64 j + t, j = 0..3, so that every child load
// instruction reads 64 consecutive floats.  A pooling window's outer columns
// come from the neighbouring lanes (lane 63's right neighbour is lane 0 of
// the next block, or the halo column X0 + 256), and the lanes of odd t, which
// hold the even (centre) columns 2u, produce pooled column u.  Same sums,
// same comparisons as the 4-columns-per-lane form.
struct CoBuf {
    float v[4][4];   // [child][block]
    float hv[4];     // halo column, per child
};

__device__ inline void load_row_co(const StreamArgs& a, const float* prev, const float* const cmap[4], int y, int X0,
                                   int t, CoBuf& b) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int yy = y + 2 * (k >> 1) - 1, dx = 2 * (k & 1) - 1;
        const bool rok = cmap[k] != nullptr && yy >= 0 && yy < a.h;     // uniform over the wave
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(rok ? cmap[k] + (size_t)yy * a.w : prev, rok ? a.w * 4 : 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = X0 + 64 * j + t + dx;   // >= -2; right of the row: past the descriptor's size
            b.v[k][j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, c >= 0 ? c * 4 : kOOB, 0, 0));
        }
        b.hv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (X0 + 256 + dx) * 4, 0, 0));
    }
}

// Horizontal first maxima (value, mx code 0..2) of the windows centred on the
// lane's four columns (meaningful on lanes of odd t).
__device__ inline void pool_row_co(const StreamArgs& a, const CoBuf& b, float inv, int y, int X0, int t, float hv[4],
                                   int hk[4]) {
    const bool yin = y >= 0 && y < a.h;
    float av[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float s = (((0.f + b.v[0][j]) + b.v[1][j]) + b.v[2][j]) + b.v[3][j];
        const float m = s * inv;
        const int x = X0 + 64 * j + t;
        av[j] = (yin && x >= 0 && x < a.w) ? fmaxf(m, 0.f) : -1.f;
    }
    float halo;
    {
        const float s = (((0.f + b.hv[0]) + b.hv[1]) + b.hv[2]) + b.hv[3];
        const float m = s * inv;
        halo = (yin && X0 + 256 < a.w) ? fmaxf(m, 0.f) : -1.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // wave_shr:1 gives lane t the value of lane t - 1 (lane 0: unused);
        // wave_shl:1 gives lane t that of lane t + 1, and lane 63, which has
        // no source lane, keeps the old operand: the next block's lane 0.
        const float nxt = j < 3 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(av[j < 3 ? j + 1 : j]), 0))
                                : halo;
        const float v0 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(av[j]), 0x138, 0xF, 0xF, false));
        const float v2 =
            __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(nxt), __float_as_int(av[j]), 0x130, 0xF, 0xF, false));
        const float v1 = av[j];
        float best = v0;
        int k = 0;
        if (v1 > best) { best = v1; k = 1; }
        if (v2 > best) { best = v2; k = 2; }
        hv[j] = best;
        hk[j] = k;
    }
}

__device__ __forceinline__ void level_coalesced_body(const StreamArgs& a, const float* __restrict__ prev,
                                            const float* const cmap[4], float inv, int P, int band, int ct, int t,
                                            float lam, float* __restrict__ cp, uint8_t* __restrict__ code) {
    const int R0 = band * a.TRo, R1 = min(R0 + a.TRo, a.hp);
    const int C0 = ct * kStreamCols, ncol = min(kStreamCols, a.wp - C0);
    const int X0 = 2 * C0 - 1;
    CoBuf b0, b1;
    float pv[4], hv[4];
    int pk[4], hk[4];
    load_row_co(a, prev, cmap, 2 * R0 - 1, X0, t, b0);
    load_row_co(a, prev, cmap, 2 * R0, X0, t, b1);
    pool_row_co(a, b0, inv, 2 * R0 - 1, X0, t, pv, pk);
    for (int r = R0; r < R1; ++r) {
        // b1 holds row 2r
        load_row_co(a, prev, cmap, 2 * r + 1, X0, t, b0);
        float best[4];
        int bk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) { best[j] = pv[j]; bk[j] = pk[j]; }
        pool_row_co(a, b1, inv, 2 * r, X0, t, hv, hk);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (hv[j] > best[j]) { best[j] = hv[j]; bk[j] = 3 + hk[j]; }
        load_row_co(a, prev, cmap, 2 * r + 2, X0, t, b1);   // row 2R1 is in range or masked
        pool_row_co(a, b0, inv, 2 * r + 1, X0, t, pv, pk);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (pv[j] > best[j]) { best[j] = pv[j]; bk[j] = 6 + pk[j]; }
            const int u = 32 * j + (t >> 1);   // lane t = 2i + 1 holds centre column 2 (C0 + 32 j + i)
            if ((t & 1) && u < ncol) {
                const size_t o = ((size_t)P * a.hp + r) * a.wp + C0 + u;
                cp[o] = rect_pow(best[j], lam);
                code[o] = (uint8_t)bk[j];
            }
        }
    }
}

template <int VEC, bool NARROW>
__device__ __forceinline__ void level_stream_body(const StreamArgs& a, const float* __restrict__ prev,
                                         const uint8_t* __restrict__ vt, const Geom& g, float lam,
                                         float* __restrict__ cp, uint8_t* __restrict__ code, int bid) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), t = threadIdx.x & 63;   // wave index: uniform
    const int item = bid * kStreamWaves + wv;
    if (item >= a.n_items) return;
    const int np = a.gx * a.gy;
    const int P = item % np, rest = item / np;
    const int ct = rest % a.n_ct, band = rest / a.n_ct;
    const int pb = P / a.gx, pa = P - pb * a.gx;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    if (!(vxp[pa] && vyp[pb])) return;
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    const size_t hw = (size_t)a.h * a.w;
    const float* cmap[4];
    int nx = 0, ny = 0, ex[2], ey[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int ca = child_index(a.l, pa, 2 * k - 1), cb = child_index(a.l, pb, 2 * k - 1);
        ex[k] = (ca >= 0 && ca < a.gxc && vxc[ca]) ? ca : -1;
        ey[k] = (cb >= 0 && cb < a.gyc && vyc[cb]) ? cb : -1;
        nx += ex[k] >= 0;
        ny += ey[k] >= 0;
    }
    if (nx * ny == 0) return;   // a valid parent always has a child; kept for safety
#pragma unroll
    for (int ky = 0; ky < 2; ++ky)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx)
            cmap[2 * ky + kx] =
                (ey[ky] >= 0 && ex[kx] >= 0) ? prev + (size_t)child_slot(g, a.l, ey[ky] * a.gxc + ex[kx]) * hw : nullptr;
    const float inv = 1.f / float(nx * ny);
    if constexpr (NARROW) {
        level_narrow_body<VEC>(a, prev, cmap, inv, P, band, t, lam, cp, code);
        return;
    }
    if constexpr (VEC == 0) {
        level_coalesced_body(a, prev, cmap, inv, P, band, ct, t, lam, cp, code);
        return;
    }
    const int R0 = band * a.TRo, R1 = min(R0 + a.TRo, a.hp);
    const int C0 = ct * kStreamCols, ncol = min(kStreamCols, a.wp - C0);
    const int X0 = 2 * C0 - 1;

    RowBuf b0, b1;
    float pv[2], hv[2];
    int pk[2], hk[2];
    load_row<VEC>(a, prev, cmap, 2 * R0 - 1, X0, t, b0);
    load_row<VEC>(a, prev, cmap, 2 * R0, X0, t, b1);
    pool_row(a, b0, inv, 2 * R0 - 1, X0, t, pv, pk);
    for (int r = R0; r < R1; ++r) {
        // b1 holds row 2r
        load_row<VEC>(a, prev, cmap, 2 * r + 1, X0, t, b0);
        float best[2];
        int bk[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) { best[q] = pv[q]; bk[q] = pk[q]; }
        pool_row(a, b1, inv, 2 * r, X0, t, hv, hk);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (hv[q] > best[q]) { best[q] = hv[q]; bk[q] = 3 + hk[q]; }
        load_row<VEC>(a, prev, cmap, 2 * r + 2, X0, t, b1);   // row 2R1 is in range or masked
        pool_row(a, b0, inv, 2 * r + 1, X0, t, pv, pk);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (pv[q] > best[q]) { best[q] = pv[q]; bk[q] = 6 + pk[q]; }
            const int u = 2 * t + q;
            if (u < ncol) {
                const size_t o = ((size_t)P * a.hp + r) * a.wp + C0 + u;
                cp[o] = rect_pow(best[q], lam);
                code[o] = (uint8_t)bk[q];
            }
        }
    }
}

template <typename T>
__device__ inline void level_top_body(const LevelArgs& a, const T* __restrict__ prev, const uint8_t* __restrict__ vt,
                                      const Geom& g, T lam, T* __restrict__ top, int bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ParentLDS<T>* sp = (ParentLDS<T>*)smem_raw;
    const int rest = bid / a.n_pblk, pblk = bid - rest * a.n_pblk;   // once per block (scalar)
    const int ct = rest / a.n_rt, R0 = (rest - ct * a.n_rt) * a.TRo, C0 = ct * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    load_parents<T>(a, g, pblk * a.PB, vxp, vyp, vxc, vyc, prev, sp);
    __syncthreads();
    for (int e = threadIdx.x; e < a.PB * a.TRo * a.TCo; e += 256) {
        const int k = fdiv(e, a.f_tile), rem = e - k * (a.TRo * a.TCo);
        const int orow = fdiv(rem, a.f_tco);
        const int qy = R0 + orow, qx = C0 + rem - orow * a.TCo;
        const int P = pblk * a.PB + k;
        if (P >= a.gx * a.gy || qy >= a.h || qx >= a.w) continue;
        // maps of non-existing top patches are written as zeros
        const T A = sp[k].valid ? staged_aggregate(a, sp[k], prev, qy, qx) : T(0);
        top[((size_t)P * a.h + qy) * a.w + qx] = rect_pow(A, lam);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_pool(LevelArgs a, const T* __restrict__ prev,
                                                    const uint8_t* __restrict__ vt, Geom g, T lam,
                                                    T* __restrict__ cp, uint8_t* __restrict__ code, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    level_pool_body<T>(a, prev, vt, g, lam, cp, code, bid);
}

template <int VEC, bool NARROW>
__global__ __launch_bounds__(64 * kStreamWaves) void k_level_stream(StreamArgs a, const float* __restrict__ prev,
                                                                     const uint8_t* __restrict__ vt, Geom g, float lam,
                                                                     float* __restrict__ cp,
                                                                     uint8_t* __restrict__ code, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    level_stream_body<VEC, NARROW>(a, prev, vt, g, lam, cp, code, bid);
}

template <typename T>
__global__ __launch_bounds__(256) void k_level_top(LevelArgs a, const T* __restrict__ prev,
                                                   const uint8_t* __restrict__ vt, Geom g, T lam,
                                                   T* __restrict__ top, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    level_top_body<T>(a, prev, vt, g, lam, top, bid);
}

struct LevelPoolJob {
    LevelArgs a;
    const float* prev;
    const uint8_t* vt;
    Geom g;
    float lam;
    float* cp;
    uint8_t* code;
    static __device__ void run(const LevelPoolJob& j, int v) {
        level_pool_body<float>(j.a, j.prev, j.vt, j.g, j.lam, j.cp, j.code, v);
    }
};

struct LevelTopJob {
    LevelArgs a;
    const float* prev;
    const uint8_t* vt;
    Geom g;
    float lam;
    float* top;
    static __device__ void run(const LevelTopJob& j, int v) {
        level_top_body<float>(j.a, j.prev, j.vt, j.g, j.lam, j.top, v);
    }
};

template <int VEC, bool NARROW>
struct LevelStreamJob {
    StreamArgs a;
    const float* prev;
    const uint8_t* vt;
    Geom g;
    float lam;
    float* cp;
    uint8_t* code;
    static __device__ void run(const LevelStreamJob& j, int v) {
        level_stream_body<VEC, NARROW>(j.a, j.prev, j.vt, j.g, j.lam, j.cp, j.code, v);
    }
};

// Tiled form of level l: the launch arguments, block count and LDS bytes.
template <typename T>
LevelArgs make_level_args(int l, const Geom& g, int& nblocks, size_t& smem) {
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
    nblocks = a.n_pblk * a.n_rt * n_ct;
    a.f_ra = make_fastdiv((2 * a.TRo + 1) * (2 * a.TCo + 1));
    a.f_rw = make_fastdiv(2 * a.TCo + 1);
    a.f_tile = make_fastdiv(a.TRo * a.TCo);
    a.f_tco = make_fastdiv(a.TCo);
    const size_t sp_bytes = ((size_t)a.PB * sizeof(ParentLDS<T>) + 15) & ~size_t(15);
    smem = is_top ? sp_bytes : sp_bytes + (size_t)a.PB * (2 * a.TRo + 1) * (2 * a.TCo + 1) * sizeof(T);
    return a;
}

// Streaming form of level l with bands of tro pooled rows.
StreamArgs make_stream_args(int l, const Geom& g, int tro, int& nblocks) {
    StreamArgs b;
    b.l = l;
    b.gx = g.gx[l];
    b.gy = g.gy[l];
    b.gxc = g.gx[l - 1];
    b.gyc = g.gy[l - 1];
    b.h = g.h[l];
    b.w = g.w[l];
    b.hp = g.h[l + 1];
    b.wp = g.w[l + 1];
    b.TRo = b.hp < tro ? b.hp : tro;
    b.n_band = (b.hp + b.TRo - 1) / b.TRo;
    b.n_ct = (b.wp + kStreamCols - 1) / kStreamCols;
    b.vec = (b.w % 4) == 0 ? 2 : ((b.w % 2) == 0 ? 1 : 0);
    // Narrow maps: one wave walks G = 64 / L bands (groups of bands per
    // item); each child's descriptor spans its whole map, whose byte size
    // must fit an int.
    b.narrow = b.vec && b.wp <= kStreamCols / 2 && (double)b.h * b.w * 4 < 2.0e9;
    b.lgl = 5;
    if (b.narrow) {   // groups of G bands of at most tro rows, the rows split evenly over the groups
        while (b.lgl > 0 && 2 * (1 << (b.lgl - 1)) >= b.wp) --b.lgl;   // smallest L with 2 L >= wp
        const int G = 64 >> b.lgl;
        b.n_band = (b.hp + G * b.TRo - 1) / (G * b.TRo);
        b.TRo = (b.hp + G * b.n_band - 1) / (G * b.n_band);
    }
    b.n_items = b.gx * b.gy * b.n_ct * b.n_band;
    nblocks = (b.n_items + kStreamWaves - 1) / kStreamWaves;
    return b;
}

// The streaming form serves FP32 levels below the top whose pooled maps are
// at least 32 columns wide, or at least 16 wide with maps a multiple of 4
// wide (the narrow form; on smaller maps a wave has too little to do and the
// tiled form is as fast).
inline bool use_stream(int l, const Geom& g) {
    return l < g.lmax && (g.w[l + 1] >= 32 || (g.w[l + 1] >= 16 && g.w[l] % 4 == 0));
}

}  // namespace

JobRec level_job(int l, const float* prev, const uint8_t* vt, const Geom& g, float lam, float* cp, uint8_t* code,
                 float* top, int tro) {
    JobRec r;
    if (use_stream(l, g)) {
        int nb;
        const StreamArgs b = make_stream_args(l, g, tro, nb);
        if (b.narrow && b.vec == 2) r.set(JK_LEVEL_NARROW, nb, 0, LevelStreamJob<2, true>{b, prev, vt, g, lam, cp, code});
        else if (b.narrow) r.set(JK_LEVEL_NARROW8, nb, 0, LevelStreamJob<1, true>{b, prev, vt, g, lam, cp, code});
        else if (b.vec == 2) r.set(JK_LEVEL_STREAM_VEC, nb, 0, LevelStreamJob<2, false>{b, prev, vt, g, lam, cp, code});
        else if (b.vec == 1) r.set(JK_LEVEL_STREAM_VEC8, nb, 0, LevelStreamJob<1, false>{b, prev, vt, g, lam, cp, code});
        else r.set(JK_LEVEL_STREAM, nb, 0, LevelStreamJob<0, false>{b, prev, vt, g, lam, cp, code});
        return r;
    }
    int nb;
    size_t smem;
    const LevelArgs a = make_level_args<float>(l, g, nb, smem);
    if (l == g.lmax) r.set(JK_LEVEL_TOP, nb, smem, LevelTopJob{a, prev, vt, g, lam, top});
    else r.set(JK_LEVEL_POOL, nb, smem, LevelPoolJob{a, prev, vt, g, lam, cp, code});
    return r;
}

hipError_t launch_group_level(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_LEVEL_STREAM_VEC: return launch_grouped<LevelStreamJob<2, false>, 64 * kStreamWaves, 1>(gl, s);
        case JK_LEVEL_STREAM_VEC8: return launch_grouped<LevelStreamJob<1, false>, 64 * kStreamWaves, 1>(gl, s);
        case JK_LEVEL_STREAM: return launch_grouped<LevelStreamJob<0, false>, 64 * kStreamWaves, 1>(gl, s);
        case JK_LEVEL_NARROW: return launch_grouped<LevelStreamJob<2, true>, 64 * kStreamWaves, 1>(gl, s);
        case JK_LEVEL_NARROW8: return launch_grouped<LevelStreamJob<1, true>, 64 * kStreamWaves, 1>(gl, s);
        case JK_LEVEL_POOL: return launch_grouped<LevelPoolJob, 256, 1>(gl, s);
        case JK_LEVEL_TOP: return launch_grouped<LevelTopJob, 256, 1>(gl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_level(int l, const T* prev, const uint8_t* vt, const Geom& g, T lam, T* cp, uint8_t* code,
                        T* top, hipStream_t s) {
    if (std::is_same<T, float>::value && use_stream(l, g)) {
        int nb;
        const StreamArgs b = make_stream_args(l, g, 16, nb);
        const float* pf = reinterpret_cast<const float*>(prev);
        float* cf = reinterpret_cast<float*>(cp);
        const dim3 grid(((nb + 7) / 8) * 8);
#define DM_LEVEL_STREAM(V, N)                                                                                      \
    hipLaunchKernelGGL((k_level_stream<V, N>), grid, dim3(64 * kStreamWaves), 0, s, b, pf, vt, g, (float)lam, cf, \
                       code, nb)
        if (b.narrow && b.vec == 2) DM_LEVEL_STREAM(2, true);
        else if (b.narrow) DM_LEVEL_STREAM(1, true);
        else if (b.vec == 2) DM_LEVEL_STREAM(2, false);
        else if (b.vec == 1) DM_LEVEL_STREAM(1, false);
        else DM_LEVEL_STREAM(0, false);
#undef DM_LEVEL_STREAM
        return hipGetLastError();
    }
    int nblocks;
    size_t smem;
    const LevelArgs a = make_level_args<T>(l, g, nblocks, smem);
    const dim3 grid(((nblocks + 7) / 8) * 8);
    if (l == g.lmax)
        hipLaunchKernelGGL(k_level_top<T>, grid, dim3(256), smem, s, a, prev, vt, g, lam, top, nblocks);
    else
        hipLaunchKernelGGL(k_level_pool<T>, grid, dim3(256), smem, s, a, prev, vt, g, lam, cp, code, nblocks);
    return hipGetLastError();
}

template hipError_t launch_level<float>(int, const float*, const uint8_t*, const Geom&, float, float*, uint8_t*,
                                        float*, hipStream_t);
template hipError_t launch_level<double>(int, const double*, const uint8_t*, const Geom&, double, double*,
                                         uint8_t*, double*, hipStream_t);

}  // namespace dm
