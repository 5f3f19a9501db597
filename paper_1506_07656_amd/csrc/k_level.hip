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
__device__ inline void load_parents(const LevelArgs& a, int pbase, const uint8_t* vxp, const uint8_t* vyp,
                                    const uint8_t* vxc, const uint8_t* vyc, const T* prev, ParentLDS<T>* sp) {
    const size_t hw = (size_t)a.h * a.w;
    for (int k = threadIdx.x; k < a.PB; k += blockDim.x) {
        const Parent<T> pi = parent_info<T>(a, pbase + k, vxp, vyp, vxc, vyc);
        ParentLDS<T> r;
#pragma unroll
        for (int ky = 0; ky < 2; ++ky)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx)
                r.cmap[2 * ky + kx] =
                    (pi.cb[ky] >= 0 && pi.ca[kx] >= 0) ? prev + (size_t)(pi.cb[ky] * a.gxc + pi.ca[kx]) * hw : nullptr;
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
__global__ __launch_bounds__(256) void k_level_pool(LevelArgs a, const T* __restrict__ prev,
                                                    const uint8_t* __restrict__ vt, Geom g, T lam,
                                                    T* __restrict__ cp, uint8_t* __restrict__ code, int nblocks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ParentLDS<T>* sp = (ParentLDS<T>*)smem_raw;
    T* sA = (T*)(smem_raw + ((a.PB * sizeof(ParentLDS<T>) + 15) & ~size_t(15)));
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    const int rest = bid / a.n_pblk, pblk = bid - rest * a.n_pblk;   // once per block (scalar)
    const int ct = rest / a.n_rt, R0 = (rest - ct * a.n_rt) * a.TRo, C0 = ct * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    load_parents<T>(a, pblk * a.PB, vxp, vyp, vxc, vyc, prev, sp);
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

template <typename T>
__global__ __launch_bounds__(256) void k_level_top(LevelArgs a, const T* __restrict__ prev,
                                                   const uint8_t* __restrict__ vt, Geom g, T lam,
                                                   T* __restrict__ top, int nblocks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ParentLDS<T>* sp = (ParentLDS<T>*)smem_raw;
    const int bid = xcd_block(nblocks);
    if (bid >= nblocks) return;
    const int rest = bid / a.n_pblk, pblk = bid - rest * a.n_pblk;   // once per block (scalar)
    const int ct = rest / a.n_rt, R0 = (rest - ct * a.n_rt) * a.TRo, C0 = ct * a.TCo;
    const uint8_t *vxp = vtab(vt, g, a.l, 0), *vyp = vtab(vt, g, a.l, 1);
    const uint8_t *vxc = vtab(vt, g, a.l - 1, 0), *vyc = vtab(vt, g, a.l - 1, 1);
    load_parents<T>(a, pblk * a.PB, vxp, vyp, vxc, vyc, prev, sp);
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
    const int nblocks = a.n_pblk * a.n_rt * n_ct;
    a.f_ra = make_fastdiv((2 * a.TRo + 1) * (2 * a.TCo + 1));
    a.f_rw = make_fastdiv(2 * a.TCo + 1);
    a.f_tile = make_fastdiv(a.TRo * a.TCo);
    a.f_tco = make_fastdiv(a.TCo);
    const dim3 grid(((nblocks + 7) / 8) * 8);
    const size_t sp_bytes = ((size_t)a.PB * sizeof(ParentLDS<T>) + 15) & ~size_t(15);
    if (is_top) {
        hipLaunchKernelGGL(k_level_top<T>, grid, dim3(256), sp_bytes, s, a, prev, vt, g, lam, top, nblocks);
    } else {
        const size_t smem = sp_bytes + (size_t)a.PB * (2 * a.TRo + 1) * (2 * a.TCo + 1) * sizeof(T);
        hipLaunchKernelGGL(k_level_pool<T>, grid, dim3(256), smem, s, a, prev, vt, g, lam, cp, code, nblocks);
    }
    return hipGetLastError();
}

template hipError_t launch_level<float>(int, const float*, const uint8_t*, const Geom&, float, float*, uint8_t*,
                                        float*, hipStream_t);
template hipError_t launch_level<double>(int, const double*, const uint8_t*, const Geom&, double, double*,
                                         uint8_t*, double*, hipStream_t);

}  // namespace dm
