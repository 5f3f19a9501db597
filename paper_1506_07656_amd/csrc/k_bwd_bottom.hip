// Adjoint of the bottom correlation (Eq. (3)) for the gradient pass.
//
// With g'_0(p, r) the gradient routed to pooled entry r of atomic patch p
// (see k_backward.hip), the gradient with respect to A_0 is
//   dA_0(p, x) = sum_{r: 2r + m_0(p, r) = x} g'_0(p, r)        (<= 4 candidates)
// and, with K index k = (dy, dx, c) over the 4x4 patch and 9 channels,
//   dD1[p + d_k][c_k] = 1/16 sum_x dA_0(p, x) D2[x + d_k][c_k]          (GEMM 1)
//   T[k][x]           =      sum_p D1[p + d_k][c_k] dA_0(p, x)          (GEMM 2)
//   dD2[y][c]         = 1/16 sum_{dy,dx} T[(d, c)][y - d]               (col2im)
// Atomic patches do not overlap, so GEMM 1 writes each D1 pixel once.
//
// Matrix-core path (FP32 or BF16 operands, FP32 accumulation): dA_0 never
// goes to memory.  Every GEMM tile stages the pooled cells (g'_0 and codes)
// its dA_0 block depends on into LDS and gathers the block there: a 2 x 2
// square of target positions (2t + i, 2u + e) receives only from the pooled
// cells (t, u), (t, u + 1), (t + 1, u), (t + 1, u + 1), each of which sends
// its value to the one position its code names, so every dA_0 entry is the
// sum of at most four staged values, added in the fixed order of (row,
// column) of the cell (deterministic).  Target positions live on a padded
// Hp x Wp grid (Wp = W' rounded up to 64, Hp = H' rounded up to 4): padding
// positions receive nothing (the forward pool never selects a position
// outside I') and read zero descriptors, so tiles never check bounds.
//  - GEMM 1 (M = 128 patches, N = 144, K = positions split over blocks): a
//    K chunk is 2 position rows x CW columns; the im2col operand of D2 is
//    stored transposed ([144][positions]) in that chunk order, contiguous
//    along K.
//  - GEMM 2 (M = 144, N = a tile of 4 position rows x 32 columns, K =
//    patches): the dA_0 chunk is gathered straight into LDS as
//    [position][patch]; the transposed patch matrix of D1 ([144][Pp], its
//    columns in the gather's patch order) is copied as it is.
// The staged cells sit in LDS in a layout that lets a lane read a run of four
// cells of a row with one 16-byte load, and each gather task turns two such
// runs (pooled rows t, t + 1) into four quads (16 target positions).
// Loads of the next chunk are in flight during the matrix-core work; split
// partial sums are added in a fixed order.
//
// Reference kernels (thread per output, direct loops) serve the FP64
// instantiation used by the finite-difference check.
#include <type_traits>

#include "dm_group.h"

namespace dm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
// Native 16-byte vector: copies are plain loads and stores, never memcpy of a
// struct, so arrays of them stay in registers.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct BotArgs {
    int W1, H1, W2, H2, n0x, natom, h1, w1;
    int Wp, H2p, Xp, Pp;   // padded target grid and patch count (matrix-core path)
    int pm;                // h1 * w1: cells of one patch's pooled map
};

// dA_0(p, x) from the pooled gradient and codes of patch p (maps h1 x w1).
template <typename T>
__device__ inline T dA_at(const T* __restrict__ gp, const uint8_t* __restrict__ code, int h1, int w1, int xy,
                          int xx) {
    T acc = 0;
    for (int ry = (xy - 1) >> 1; ry <= (xy + 1) >> 1; ++ry) {
        const int my = xy - 2 * ry;
        if (ry < 0 || ry >= h1 || my < -1 || my > 1) continue;
        for (int rx = (xx - 1) >> 1; rx <= (xx + 1) >> 1; ++rx) {
            const int mx = xx - 2 * rx;
            if (rx < 0 || rx >= w1 || mx < -1 || mx > 1) continue;
            const int o = ry * w1 + rx;
            if (code[o] == 3 * (my + 1) + (mx + 1)) acc += gp[o];
        }
    }
    return acc;
}

// im2col entries: target descriptor at position x shifted by patch offset k.
template <typename T>
__device__ inline T d2_at(const T* __restrict__ d2, const BotArgs& a, int xy, int xx, int k) {
    const int dy = k / 36, dx = (k / 9) % 4, c = k % 9;
    const int y = xy - 2 + dy, x = xx - 2 + dx;
    return (y >= 0 && y < a.H2 && x >= 0 && x < a.W2) ? d2[((size_t)y * a.W2 + x) * 9 + c] : T(0);
}
template <typename T>
__device__ inline T d1_at(const T* __restrict__ d1, const BotArgs& a, int p, int k) {
    const int b = p / a.n0x, aa = p - b * a.n0x;
    const int dy = k / 36, dx = (k / 9) % 4, c = k % 9;
    return d1[((size_t)(4 * b + dy) * a.W1 + 4 * aa + dx) * 9 + c];
}

__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline bf8 as_bf8(const uint16_t* p) {   // 8 consecutive bf16 (16-byte aligned)
    union {
        uint4 u;
        bf8 v;
    } x;
    x.u = *(const uint4*)p;
    return x.v;
}

// 8 values -> one 16-byte (BF16) or two 16-byte (FP32) stores.
template <typename E>
__device__ inline void store8(E* dst, const float v[8]) {
    if constexpr (std::is_same<E, float>::value) {
        reinterpret_cast<float4*>(dst)[0] = make_float4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<float4*>(dst)[1] = make_float4(v[4], v[5], v[6], v[7]);
    } else {
        uint4 u;
        u.x = (uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
        u.y = (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
        u.z = (uint32_t)to_bf16(v[4]) | ((uint32_t)to_bf16(v[5]) << 16);
        u.w = (uint32_t)to_bf16(v[6]) | ((uint32_t)to_bf16(v[7]) << 16);
        *reinterpret_cast<uint4*>(dst) = u;
    }
}

constexpr int kPadW = 64, kPadH = 4;   // target grid padding (columns, rows)

// ---------------------------------------------------------------- staging and gather
constexpr int kOOB = 0x7ffffff0;   // buffer byte offset past any map

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

// LDS image of the pooled cells of NP patches (from patch p0), pooled rows
// r0 .. r0 + NR - 1 and columns s0 .. s0 + NM (NM a multiple of 4).
//  - main[p][r][0 .. NM): patch stride S with S % 8 == 4, so that lanes
//    taking consecutive patches read their 16-byte runs of a row on distinct
//    banks;
//  - column NM as xcol[r][p] (consecutive patches in consecutive words), and
//    with DUP the columns 4, 8, ..., NM - 4 once more beside it
//    (dup[c / 4 - 1][r][p]): the cell after a lane's run of four, read
//    without conflicts.  Without DUP a lane takes that cell from the lane
//    that holds the next run (run5_lanes).
// BF16: one word per cell, the value in the high half and the code in the
// low byte (the staged value is the BF16 gradient itself); FP32: a value word
// and a code byte at the same index.
// Loading: thread t keeps column t % NM of the first NM columns, and u =
// t / NM picks its first (patch, row); its k-th cell is u + (256 / NM) k in
// (patch, row) order for two rows (row fastest: the lanes of a store then
// cover 32 banks) and in (row, patch) order otherwise, so every offset is the
// thread's base plus a stride known at compile time, and the lanes of a load
// read runs of NM neighbouring cells of a row.  Column NM goes to the threads
// in (row, patch) order.  Values wait in registers between their loads and
// their LDS store: BF16 values with their codes in one register, FP32 values
// beside codes packed four to a register.  Cells outside the map or the patch
// range are 0 (value and code): they add nothing.  One buffer descriptor
// starts at patch p0; the host keeps 128 x h1 x w1 x 4 bytes below 2^31, so
// every offset fits.
template <bool BF16, int NP, int NR, int NM, bool DUP>
struct CellImage {
    static_assert(NM % 4 == 0 && 256 % NM == 0, "runs of four cells; whole rows per pass");
    static constexpr int RPK = 256 / NM;                  // rows of NM cells one pass covers
    static constexpr bool RFAST = NR == 2;
    static_assert(RFAST ? RPK % 2 == 0 : NP % RPK == 0, "a thread keeps its row");
    static constexpr int PM = NP * NR * NM / 256;         // first-NM-column cells per thread
    static constexpr int NX = NP * NR, PX = (NX + 255) / 256;   // column-NM cells (per thread)
    static constexpr int CM = BF16 ? PM : (PM + 3) / 4, CX = BF16 ? PX : (PX + 3) / 4;
    static constexpr int S = NR * NM + ((NR * NM) % 8 == 4 ? 0 : 4);
    static constexpr int D0 = NP * S;                              // start of dup
    static constexpr int X0 = D0 + (DUP ? (NM / 4 - 1) * NR * NP : 0);   // start of xcol
    static constexpr int WORDS = X0 + NR * NP;            // image words (FP32: as many code bytes)
    // row and patch of cell k of a thread, beyond those of its first cell
    static constexpr int kr(int k) { return RFAST ? 0 : RPK * k / NP; }
    static constexpr int kp(int k) { return RFAST ? RPK / 2 * k : RPK * k % NP; }
    __device__ static __forceinline__ int row0() { return RFAST ? (int)(threadIdx.x / NM) % 2 : 0; }
    __device__ static __forceinline__ int patch0() {
        return RFAST ? (int)(threadIdx.x / NM) / 2 : (int)(threadIdx.x / NM);
    }
    uint32_t vm[PM], vx[PX];   // values (BF16: the 16 bits)
    uint32_t cm[CM], cx[CX];   // codes (BF16: one per register; FP32: four to a word)

    __device__ __forceinline__ void load(const void* __restrict__ gp, const uint8_t* __restrict__ code,
                                         const BotArgs& a, int p0, int r0, int s0) {
        constexpr int es = BF16 ? 2 : 4;
        const uint32_t pm = (uint32_t)a.pm;
        // patches of this range that exist (none when p0 is past the last one)
        const uint32_t np = p0 < a.natom ? (uint32_t)min(NP, a.natom - p0) : 0u;
        const auto rsG = buf_rsrc(static_cast<const char*>(gp) + (size_t)p0 * pm * es, np * pm * es);
        const auto rsM = buf_rsrc(code + (size_t)p0 * pm, np * pm);
        const int col = threadIdx.x % NM, rt = row0();
        // element offset of the thread's first cell; cell k adds the uniform kp(k) pm + kr(k) w1
        const uint32_t o0 = (uint32_t)patch0() * pm + (uint32_t)(r0 + rt) * a.w1 + s0 + col;
        auto put = [&](uint32_t* v, uint32_t* c, int k, uint32_t om, uint32_t og) {
            const uint32_t m = __builtin_amdgcn_raw_buffer_load_b8(rsM, (int)om, 0, 0);
            // BF16 keeps value and code apart until the LDS store: joining
            // them here would wait for the loads.
            if constexpr (BF16) {
                v[k] = __builtin_amdgcn_raw_buffer_load_b16(rsG, (int)og, 0, 0);
                c[k] = m;
            } else {
                v[k] = __builtin_amdgcn_raw_buffer_load_b32(rsG, (int)og, 0, 0);
                if (k % 4 == 0) c[k / 4] = m;
                else c[k / 4] |= m << (8 * (k % 4));
            }
        };
        if (r0 + NR <= a.h1 && s0 + NM + 1 <= a.w1) {   // uniform: no cell leaves the map
            const uint32_t ob = o0 * es;
#pragma unroll
            for (int k = 0; k < PM; ++k) {
                const uint32_t d = (uint32_t)kp(k) * pm + (uint32_t)kr(k) * a.w1;   // uniform
                put(vm, cm, k, o0 + d, ob + d * es);
            }
        } else {
            const bool colok = s0 + col < a.w1;
#pragma unroll
            for (int k = 0; k < PM; ++k) {
                const bool ok = colok && r0 + rt + kr(k) < a.h1;
                const uint32_t o = ok ? o0 + (uint32_t)kp(k) * pm + (uint32_t)kr(k) * a.w1 : (uint32_t)(kOOB / es);
                put(vm, cm, k, o, o * es);
            }
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int e = threadIdx.x + 256 * k, r = e / NP, p = e - r * NP;
            const bool ok = e < NX && s0 + NM < a.w1 && r0 + r < a.h1;
            const uint32_t o = ok ? (uint32_t)p * pm + (uint32_t)(r0 + r) * a.w1 + s0 + NM : (uint32_t)(kOOB / es);
            put(vx, cx, k, o, o * es);
        }
    }
    __device__ __forceinline__ void store(uint32_t* __restrict__ img, uint8_t* __restrict__ cimg) const {
        const int col = threadIdx.x % NM, rt = row0(), pt = patch0();
        const int mi = pt * S + rt * NM + col;
        const bool dup = DUP && col > 0 && col % 4 == 0;
        const int di = D0 + ((col / 4 - 1) * NR + rt) * NP + pt;
        auto put = [&](int slot, uint32_t v, const uint32_t* c, int k) {
            if constexpr (BF16) {
                img[slot] = (v << 16) | c[k];
            } else {
                img[slot] = v;
                cimg[slot] = (uint8_t)(c[k / 4] >> (8 * (k % 4)));
            }
        };
#pragma unroll
        for (int k = 0; k < PM; ++k) {
            put(mi + kp(k) * S + kr(k) * NM, vm[k], cm, k);
            if (dup) put(di + kr(k) * NP + kp(k), vm[k], cm, k);
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int e = threadIdx.x + 256 * k;
            if (NX % 256 == 0 || e < NX) put(X0 + e, vx[k], cx, k);
        }
    }
    __device__ static __forceinline__ void decode(uint32_t w, uint32_t cb, float& g, int& m) {
        if constexpr (BF16) {
            g = __uint_as_float(w & 0xFFFF0000u);
            m = (int)(w & 0xFFu);
        } else {
            g = __uint_as_float(w);
            m = (int)cb;
        }
    }
    // Cells (r, 4 q4 .. 4 q4 + 4) of patch p (DUP): values g and codes m.
    __device__ static __forceinline__ void run5(const uint32_t* __restrict__ img, const uint8_t* __restrict__ cimg,
                                                int p, int r, int q4, float g[5], int m[5]) {
        static_assert(DUP, "the cell after a run comes from dup");
        const int mi = p * S + r * NM + 4 * q4;
        const int di = (q4 + 1) * 4 == NM ? X0 + r * NP + p : D0 + (q4 * NR + r) * NP + p;
        const u32x4 w = *reinterpret_cast<const u32x4*>(img + mi);
        const uint32_t cw = BF16 ? 0u : *reinterpret_cast<const uint32_t*>(cimg + mi);
#pragma unroll
        for (int j = 0; j < 4; ++j) decode(w[j], (cw >> (8 * j)) & 0xFFu, g[j], m[j]);
        decode(img[di], BF16 ? 0u : cimg[di], g[4], m[4]);
    }
    // The same for BF16 without DUP when the 64 lanes of the wave take runs
    // q4 = lane / 16 of 16 patches (NM = 16): the cell after a run is the
    // first cell of the run of the lane 16 places up, and for the last run
    // the column-NM cell, which the lane of run 0 sends (64 lanes wrap).
    __device__ static __forceinline__ void run5_lanes(const uint32_t* __restrict__ img, int p, int r, int q4,
                                                      float g[5], int m[5]) {
        static_assert(BF16 && !DUP && NM == 16, "four runs over the 64 lanes");
        const u32x4 w = *reinterpret_cast<const u32x4*>(img + p * S + r * NM + 4 * q4);
        const uint32_t xc = img[X0 + r * NP + p];   // read by every lane: no branch around it
        const uint32_t send = q4 == 0 ? xc : w[0];
        const int src = (((int)threadIdx.x & 63) + 16) & 63;
        const uint32_t nx = (uint32_t)__builtin_amdgcn_ds_bpermute(src * 4, (int)send);
#pragma unroll
        for (int j = 0; j < 4; ++j) decode(w[j], 0u, g[j], m[j]);
        decode(nx, 0u, g[4], m[4]);
    }
};

// The 2 x 2 target positions (2t + i, 2u + e), i, e in {0, 1}, from the four
// pooled cells c[di][dj] = (t + di, u + dj): value g, code m = 3(my+1)+(mx+1);
// cell (t + di, u + dj) sends to (2(t + di) + my, 2(u + dj) + mx).
__device__ __forceinline__ void gather_quad(const float g[2][2], const int m[2][2], float o[2][2]) {
    o[0][0] = m[0][0] == 4 ? g[0][0] : 0.f;
    o[0][1] = (m[0][0] == 5 ? g[0][0] : 0.f) + (m[0][1] == 3 ? g[0][1] : 0.f);
    o[1][0] = (m[0][0] == 7 ? g[0][0] : 0.f) + (m[1][0] == 1 ? g[1][0] : 0.f);
    o[1][1] = (m[0][0] == 8 ? g[0][0] : 0.f) + (m[0][1] == 6 ? g[0][1] : 0.f) + (m[1][0] == 2 ? g[1][0] : 0.f) +
              (m[1][1] == 0 ? g[1][1] : 0.f);
}

// Four neighbouring quads: pooled rows t, t + 1, cells u0 .. u0 + 4 of each
// (g0/m0 and g1/m1) -> target rows 2t and 2t + 1, positions 2 u0 .. 2 u0 + 7.
__device__ __forceinline__ void gather_run(const float g0[5], const int m0[5], const float g1[5], const int m1[5],
                                           float o[2][8]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float gv[2][2] = {{g0[q], g0[q + 1]}, {g1[q], g1[q + 1]}};
        const int mv[2][2] = {{m0[q], m0[q + 1]}, {m1[q], m1[q + 1]}};
        float oq[2][2];
        gather_quad(gv, mv, oq);
        o[0][2 * q] = oq[0][0];
        o[0][2 * q + 1] = oq[0][1];
        o[1][2 * q] = oq[1][0];
        o[1][2 * q + 1] = oq[1][1];
    }
}

// Round to nearest even, two values to one word (lo in the low half).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const bf2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// ---------------------------------------------------------------- GEMMs
// GEMM 1 shapes: 128 patches per block; K chunk = 2 position rows x CW columns.
template <bool BF16>
struct G1 {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    static constexpr int M = 128;
    static constexpr int CW = BF16 ? 32 : 16;
    static constexpr int GK = 2 * CW;
    static constexpr int NS = CW / 2 + 1;          // pooled columns a chunk reads (2 pooled rows)
    static constexpr int VPR = BF16 ? 8 : 4;       // values per 16-byte vector
    static constexpr int PAD = BF16 ? 8 : 4;       // LDS row padding (rows stay 16-byte aligned)
    static constexpr int CV = GK / VPR;            // vectors per chunk row
};
// GEMM 2 shapes: a tile of 4 position rows x 32 columns; K chunk = GK patches.
template <bool BF16>
struct G2 {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    static constexpr int TR = 4, TW = 32, N = TR * TW;
    static constexpr int GK = BF16 ? 64 : 32;
    static constexpr int NR = TR / 2 + 1, NS = TW / 2 + 1;
    static constexpr int VPR = BF16 ? 8 : 4;
    static constexpr int PAD = BF16 ? 8 : 4;
    static constexpr int CV = GK / VPR;
};

// Number of GEMM 1 K chunks of a pair and their position -> column map.
__device__ __host__ inline int g1_chunks(const BotArgs& a, int cw) { return (a.H2p / 2) * (a.Wp / cw); }
// K splits of one patch tile that run side by side (the split count is a
// multiple of it).
__device__ __host__ inline int g1_group(int nsplit) { return nsplit < 8 ? nsplit : 8; }

// C[M=128 patches][N=144] += dA_0[M][K] * D2col[N][K]^T over the chunks of one split.
template <bool BF16>
__device__ __forceinline__ void bwd_gemm1_body(const void* __restrict__ gp, const uint8_t* __restrict__ code,
                                               const typename G1<BF16>::E* __restrict__ d2colT, const BotArgs& a,
                                               int nsplit, float* __restrict__ part, int bid) {
    typedef G1<BF16> O;
    typedef typename O::E E;
    // BF16: a lane's gather task yields its A operand (below), no LDS tile.
    typedef CellImage<BF16, O::M, 2, O::CW / 2, !BF16> C;
    __shared__ __align__(16) E sA[BF16 ? 1 : O::M][O::GK + O::PAD];
    __shared__ __align__(16) E sB[144][O::GK + O::PAD];
    __shared__ __align__(16) uint32_t img[C::WORDS];
    __shared__ __align__(16) uint8_t cimg[BF16 ? 16 : C::WORDS];
    constexpr int NB = (144 * O::CV + 255) / 256;
    // Block bid = ((sg * ptiles) + ptile) * gs + m runs K split sg * gs + m of
    // patch tile ptile.  Split s takes the chunks s, s + nsplit, s + 2 nsplit,
    // ... so the gs splits of one group read neighbouring column strips of
    // the same pooled rows at the same time: they share the cache lines of
    // g'_0 and the codes, and the patch tiles beside them share the im2col
    // operand.  (One split per contiguous K range instead left each line to
    // be re-read by the same block a chunk later, after the other blocks of
    // its XCD had pushed it out of L2.)
    const int ptiles = a.Pp / O::M, gs = g1_group(nsplit);
    const int m = bid % gs, r = bid / gs, ptile = r % ptiles, split = (r / ptiles) * gs + m;
    const int nch = g1_chunks(a, O::CW), njc = a.Wp / O::CW;
    const int P0 = ptile * O::M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    // Prefetch registers for the D2col chunk, filled by unconditional loads
    // (rows past 144 are clamped and not stored) so that they stay in VGPRs.
    // Vector i of thread t is row t / CV + i (256 / CV), vector t % CV of it.
    static_assert(256 % O::CV == 0, "whole rows per pass");
    constexpr int RB = 256 / O::CV;
    u32x4 rb[NB];
    const E* const bsrc = d2colT + (size_t)(tid / O::CV) * a.Xp + (tid % O::CV) * O::VPR;
    const int bdst = (tid / O::CV) * (O::GK + O::PAD) + (tid % O::CV) * O::VPR;
    C cells;
    f4 acc[2][9];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int c) {
        const int t = c / njc, j = c - t * njc;
        cells.load(gp, code, a, P0, t, j * (O::CW / 2));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int r = min(tid / O::CV + i * RB, 143) - tid / O::CV;   // clamped row, relative
            rb[i] = *reinterpret_cast<const u32x4*>(bsrc + (size_t)r * a.Xp + (size_t)c * O::GK);
        }
    };
    if (split < nch) load(split);
    for (int c = split; c < nch; c += nsplit) {
        __syncthreads();   // the previous chunk's gather and products are done with the LDS
        cells.store(img, cimg);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (tid / O::CV + i * RB < 144) *reinterpret_cast<u32x4*>(&sB[0][0] + bdst + i * RB * (O::GK + O::PAD)) = rb[i];
        __syncthreads();
        if (c + nsplit < nch) load(c + nsplit);   // next chunk in flight during the gather and the products
        if constexpr (BF16) {
            // Lane (n, g) of wave w gathers run g of patch 32 w + 16 mt + n:
            // target rows 2t and 2t + 1, columns 8g .. 8g + 7, which are the
            // K elements 8g .. 8g + 7 of row n of the A operand for s = 0
            // and s = 1 (chunk order: K = i * CW + column).
            bf8 av[2][2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int p = wave * 32 + mt * 16 + n;
                float g0[5], g1[5], o[2][8];
                int m0[5], m1[5];
                C::run5_lanes(img, p, 0, g, g0, m0);
                C::run5_lanes(img, p, 1, g, g1, m1);
                gather_run(g0, m0, g1, m1, o);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    u32x4 w;
#pragma unroll
                    for (int j = 0; j < 4; ++j) w[j] = pack_bf16x2(o[i][2 * j], o[i][2 * j + 1]);
                    av[mt][i] = __builtin_bit_cast(bf8, w);
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const bf8 bv = as_bf8(&sB[16 * nt + n][32 * s + 8 * g]);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt][s], bv, acc[mt][nt], 0, 0, 0);
                }
        } else {
            // gather: task (patch p, run q4 of four quads) -> sA[p][i * CW + 8 q4 .. + 7];
            // consecutive lanes take consecutive patches
            constexpr int NG = O::CW / 8;
#pragma unroll
            for (int k = 0; k < O::M * NG / 256; ++k) {
                const int q = tid + 256 * k, p = q % O::M, q4 = q / O::M;
                float g0[5], g1[5], o[2][8];
                int m0[5], m1[5];
                C::run5(img, cimg, p, 0, q4, g0, m0);
                C::run5(img, cimg, p, 1, q4, g1, m1);
                gather_run(g0, m0, g1, m1, o);
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    *reinterpret_cast<float4*>(&sA[p][i * O::CW + 8 * q4]) = make_float4(o[i][0], o[i][1], o[i][2], o[i][3]);
                    *reinterpret_cast<float4*>(&sA[p][i * O::CW + 8 * q4 + 4]) =
                        make_float4(o[i][4], o[i][5], o[i][6], o[i][7]);
                }
            }
            __syncthreads();
#pragma unroll 4
            for (int t = 0; t < O::GK / 4; ++t) {
                const float a0 = sA[wave * 32 + n][4 * t + g], a1 = sA[wave * 32 + 16 + n][4 * t + g];
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const float bv = sB[16 * nt + n][4 * t + g];
                    acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv, acc[0][nt], 0, 0, 0);
                    acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv, acc[1][nt], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = P0 + wave * 32 + mt * 16 + 4 * g + j;
                if (p < a.natom) part[((size_t)split * a.natom + p) * 144 + 16 * nt + n] = acc[mt][nt][j];
            }
}

// Transposed im2col of D2 in GEMM 1's chunk order: column c * GK + i * CW + cc
// of D2colT[k] is target position (2t + i, j * CW + cc) of chunk c = t * (Wp / CW) + j.
template <bool BF16>
__device__ inline void bwd_d2col_body(const float* __restrict__ d2, const BotArgs& a,
                                      typename G1<BF16>::E* __restrict__ d2colT, int bid) {
    typedef G1<BF16> O;
    const size_t v = (size_t)bid * 256 + threadIdx.x;   // one group of 8 positions
    const int gpr = a.Xp / 8;
    if (v >= (size_t)144 * gpr) return;
    const int k = v / gpr, x0 = (int)(v - (size_t)k * gpr) * 8;
    const int c = x0 / O::GK, w = x0 - c * O::GK, i = w / O::CW, cc = w - i * O::CW;
    const int njc = a.Wp / O::CW, t = c / njc, j = c - t * njc;
    const int y = 2 * t + i, xx0 = j * O::CW + cc;
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = (y < a.H2 && xx0 + q < a.W2) ? d2_at(d2, a, y, xx0 + q, k) : 0.f;
    store8<typename O::E>(d2colT + (size_t)k * a.Xp + x0, out);
}

// Transposed patch matrix of D1: PT[k][slot] = D1[p + d_k][c_k] (0 for
// padding patches).  FP32: slot = p.  BF16: GEMM 2 gathers patches p and
// p + 32 of a 64-patch chunk into neighbouring slots 2p and 2p + 1, and the
// columns follow that order.
template <typename E>
__device__ inline void bwd_pt_body(const float* __restrict__ d1, const BotArgs& a, E* __restrict__ PT, int bid) {
    const size_t v = (size_t)bid * 256 + threadIdx.x;
    const int gpr = a.Pp / 8;
    if (v >= (size_t)144 * gpr) return;
    const int k = v / gpr, s0 = (int)(v - (size_t)k * gpr) * 8;
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int sl = s0 + q;
        const int p = std::is_same<E, float>::value ? sl : (sl & ~63) + ((sl & 63) >> 1) + 32 * (sl & 1);
        out[q] = p < a.natom ? d1_at(d1, a, p, k) : 0.f;
    }
    store8<E>(PT + (size_t)k * a.Pp + s0, out);
}

// dD1 (HWC) from the split partials: each pixel belongs to at most one patch.
template <typename T>
__device__ inline void bwd_dd1_reduce_body(const T* __restrict__ part, const BotArgs& a, int nsplit, T* __restrict__ dd1,
                                           int bid) {
    const size_t n = (size_t)a.H1 * a.W1 * 9;
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = i % 9;
    const int x = (i / 9) % a.W1, y = i / (9 * (size_t)a.W1);
    const int b = y / 4, aa = x / 4;
    T v = 0;
    if (b < a.H1 / 4 && aa < a.n0x) {
        const int p = b * a.n0x + aa;
        const int k = (y - 4 * b) * 36 + (x - 4 * aa) * 9 + c;
        for (int s = 0; s < nsplit; ++s) v += part[((size_t)s * a.natom + p) * 144 + k];
        v /= T(16);
    }
    dd1[i] = v;
}

// T[M=144][N = 4 x 32 positions] += PT[M][K] * dA_0[K][N] over all patch
// chunks; the dA_0 chunk is gathered into LDS as [position][patch].
template <bool BF16>
__device__ __forceinline__ void bwd_gemm2_body(const void* __restrict__ gp, const uint8_t* __restrict__ code,
                                               const typename G2<BF16>::E* __restrict__ PT, const BotArgs& a,
                                               float* __restrict__ tt, int bid) {
    typedef G2<BF16> O;
    typedef typename O::E E;
    typedef CellImage<BF16, O::GK, O::NR, O::TW / 2, true> C;
    __shared__ __align__(16) E sA[144][O::GK + O::PAD];   // PT chunk [k][patch slot]
    __shared__ __align__(16) E sB[O::N][O::GK + O::PAD];  // dA_0 chunk [position][patch slot]
    __shared__ __align__(16) uint32_t img[C::WORDS];
    __shared__ __align__(16) uint8_t cimg[BF16 ? 16 : C::WORDS];
    constexpr int NPT = (144 * O::CV + 255) / 256;
    const int ntw = a.Wp / O::TW;
    const int tr = bid / ntw, tc = bid - tr * ntw;
    const int Y0 = tr * O::TR, X0 = tc * O::TW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    // Vector i of thread t is row t / CV + i (256 / CV), vector t % CV of it
    // (rows past 144 are clamped and not stored).
    static_assert(256 % O::CV == 0, "whole rows per pass");
    constexpr int RB = 256 / O::CV;
    u32x4 rp[NPT];
    const E* const psrc = PT + (size_t)(tid / O::CV) * a.Pp + (tid % O::CV) * O::VPR;
    const int pdst = (tid / O::CV) * (O::GK + O::PAD) + (tid % O::CV) * O::VPR;
    C cells;
    f4 acc[9][2];
#pragma unroll
    for (int mt = 0; mt < 9; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int p0) {
        cells.load(gp, code, a, p0, Y0 / 2, X0 / 2);
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int r = min(tid / O::CV + i * RB, 143) - tid / O::CV;   // clamped row, relative
            rp[i] = *reinterpret_cast<const u32x4*>(psrc + (size_t)r * a.Pp + p0);
        }
    };
    load(0);
    // chunks past the last patch would add zeros: the walk ends at natom
    for (int p0 = 0; p0 < a.natom; p0 += O::GK) {
        __syncthreads();
        cells.store(img, cimg);
#pragma unroll
        for (int i = 0; i < NPT; ++i)
            if (tid / O::CV + i * RB < 144) *reinterpret_cast<u32x4*>(&sA[0][0] + pdst + i * RB * (O::GK + O::PAD)) = rp[i];
        __syncthreads();
        if (p0 + O::GK < a.natom) load(p0 + O::GK);
        // gather: task (patch pair pg, quad row pair rq, run q4 of four quads);
        // consecutive lanes take consecutive pairs.  BF16 pairs patches pg and
        // pg + 32 into one 32-bit word per position (patch slot 2 pg + h
        // holds patch pg + 32 h, the order of the patch matrix's columns),
        // FP32 takes one patch.
        constexpr int PG = BF16 ? 2 : 1, NPG = O::GK / PG;
        static_assert(NPG * (O::TR / 2) * (O::TW / 8) == 256, "one task per thread");
        {
            const int pg = tid % NPG, rest = tid / NPG, q4 = rest % (O::TW / 8), rq = rest / (O::TW / 8);
            float o[PG][2][8];
#pragma unroll
            for (int h = 0; h < PG; ++h) {
                float g0[5], g1[5];
                int m0[5], m1[5];
                C::run5(img, cimg, pg + NPG * h, rq, q4, g0, m0);
                C::run5(img, cimg, pg + NPG * h, rq + 1, q4, g1, m1);
                gather_run(g0, m0, g1, m1, o[h]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    const int pos = (2 * rq + i) * O::TW + 8 * q4 + x;
                    if constexpr (BF16)
                        *reinterpret_cast<uint32_t*>(&sB[pos][2 * pg]) = pack_bf16x2(o[0][i][x], o[1][i][x]);
                    else
                        sB[pos][pg] = o[0][i][x];
                }
        }
        __syncthreads();
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < O::GK / 32; ++s) {
                bf8 bv[2];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) bv[nt] = as_bf8(&sB[wave * 32 + nt * 16 + n][32 * s + 8 * g]);
#pragma unroll
                for (int mt = 0; mt < 9; ++mt) {
                    const bf8 av = as_bf8(&sA[16 * mt + n][32 * s + 8 * g]);
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[nt], acc[mt][nt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 4
            for (int t = 0; t < O::GK / 4; ++t) {
                const float b0 = sB[wave * 32 + n][4 * t + g], b1 = sB[wave * 32 + 16 + n][4 * t + g];
#pragma unroll
                for (int mt = 0; mt < 9; ++mt) {
                    const float av = sA[16 * mt + n][4 * t + g];
                    acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b0, acc[mt][0], 0, 0, 0);
                    acc[mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b1, acc[mt][1], 0, 0, 0);
                }
            }
        }
    }
    // wave w holds position row Y0 + w, columns X0 .. X0 + 31
#pragma unroll
    for (int mt = 0; mt < 9; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                tt[(size_t)(16 * mt + 4 * g + j) * a.Xp + (size_t)(Y0 + wave) * a.Wp + X0 + nt * 16 + n] =
                    acc[mt][nt][j];
}

// dD2[y][c] = 1/16 sum_d T[(d, c)][y - d] on the padded grid (T is zero outside the target).
__device__ inline void bwd_col2im_body(const float* __restrict__ tt, const BotArgs& a, float* __restrict__ dd2,
                                       int bid) {
    const size_t n = (size_t)a.H2 * a.W2 * 9;
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = i % 9;
    const int x = (i / 9) % a.W2, y = i / (9 * (size_t)a.W2);
    float v = 0.f;
    for (int dy = 0; dy < 4; ++dy) {
        const int qy = y + 2 - dy;          // position whose patch covers y at row offset dy
        if (qy < 0 || qy >= a.H2) continue;
        for (int dx = 0; dx < 4; ++dx) {
            const int qx = x + 2 - dx;
            if (qx < 0 || qx >= a.W2) continue;
            v += tt[(size_t)(dy * 36 + dx * 9 + c) * a.Xp + (size_t)qy * a.Wp + qx];
        }
    }
    dd2[i] = v / 16.f;
}

// ---------------------------------------------------------------- reference kernels
template <typename T>
__global__ void k_bwd_dd1_ref(const T* __restrict__ gp, const uint8_t* __restrict__ code, const T* __restrict__ d2,
                              BotArgs a, T* __restrict__ part) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)a.natom * 144) return;
    const int p = i / 144, k = i % 144;
    const size_t pm = (size_t)a.h1 * a.w1;
    T acc = 0;
    for (int ry = 0; ry < a.h1; ++ry)
        for (int rx = 0; rx < a.w1; ++rx) {
            const size_t o = p * pm + (size_t)ry * a.w1 + rx;
            const T gv = gp[o];
            if (gv == T(0)) continue;
            const int m = code[o];
            acc += gv * d2_at(d2, a, 2 * ry + m / 3 - 1, 2 * rx + m % 3 - 1, k);
        }
    part[i] = acc;
}

template <typename T>
__global__ void k_bwd_t_ref(const T* __restrict__ gp, const uint8_t* __restrict__ code, const T* __restrict__ d1,
                            BotArgs a, T* __restrict__ tbuf) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)a.H2 * a.W2 * 144) return;
    const int k = i % 144;
    const int xl = i / 144;
    const int xy = xl / a.W2, xx = xl % a.W2;
    const size_t pm = (size_t)a.h1 * a.w1;
    T acc = 0;
    for (int p = 0; p < a.natom; ++p) {
        const T d = dA_at(gp + p * pm, code + p * pm, a.h1, a.w1, xy, xx);
        if (d != T(0)) acc += d * d1_at(d1, a, p, k);
    }
    tbuf[i] = acc;
}

// col2im of the reference layout tbuf[x][k].
template <typename T>
__global__ void k_bwd_col2im_ref(const T* __restrict__ tbuf, BotArgs a, T* __restrict__ dd2) {
    const size_t n = (size_t)a.H2 * a.W2 * 9;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = i % 9;
    const int x = (i / 9) % a.W2, y = i / (9 * (size_t)a.W2);
    T v = 0;
    for (int dy = 0; dy < 4; ++dy) {
        const int qy = y + 2 - dy;
        if (qy < 0 || qy >= a.H2) continue;
        for (int dx = 0; dx < 4; ++dx) {
            const int qx = x + 2 - dx;
            if (qx < 0 || qx >= a.W2) continue;
            v += tbuf[((size_t)qy * a.W2 + qx) * 144 + dy * 36 + dx * 9 + c];
        }
    }
    dd2[i] = v / T(16);
}

// ---------------------------------------------------------------- kernels and jobs
// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// works through one contiguous range (GEMM 1: the K splits of a group and the
// patch tiles beside them run on one XCD and share its L2).
__device__ inline int xcd_block(int nblocks) {
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_d2col(const float* __restrict__ d2, BotArgs a,
                                                   typename G1<BF16>::E* __restrict__ d2colT) {
    bwd_d2col_body<BF16>(d2, a, d2colT, blockIdx.x);
}
template <typename E>
__global__ __launch_bounds__(256) void k_bwd_pt(const float* __restrict__ d1, BotArgs a, E* __restrict__ PT) {
    bwd_pt_body<E>(d1, a, PT, blockIdx.x);
}
template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_bwd_gemm1(const void* __restrict__ gp, const uint8_t* __restrict__ code,
                                                   const typename G1<BF16>::E* __restrict__ d2colT, BotArgs a,
                                                   int nsplit, float* __restrict__ part, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid < nblocks) bwd_gemm1_body<BF16>(gp, code, d2colT, a, nsplit, part, bid);
}
template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_bwd_gemm2(const void* __restrict__ gp, const uint8_t* __restrict__ code,
                                                   const typename G2<BF16>::E* __restrict__ PT, BotArgs a,
                                                   float* __restrict__ tt, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid < nblocks) bwd_gemm2_body<BF16>(gp, code, PT, a, tt, bid);
}
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_dd1_reduce(const T* __restrict__ part, BotArgs a, int nsplit,
                                                        T* __restrict__ dd1) {
    bwd_dd1_reduce_body<T>(part, a, nsplit, dd1, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_bwd_col2im(const float* __restrict__ tt, BotArgs a, float* __restrict__ dd2) {
    bwd_col2im_body(tt, a, dd2, blockIdx.x);
}

template <bool BF16>
struct D2colJob {
    const float* d2;
    BotArgs a;
    typename G1<BF16>::E* d2colT;
    static __device__ void run(const D2colJob& j, int v) { bwd_d2col_body<BF16>(j.d2, j.a, j.d2colT, v); }
};
template <typename E>
struct PtJob {
    const float* d1;
    BotArgs a;
    E* PT;
    static __device__ void run(const PtJob& j, int v) { bwd_pt_body<E>(j.d1, j.a, j.PT, v); }
};
template <bool BF16>
struct Gemm1Job {
    const void* gp;
    const uint8_t* code;
    const typename G1<BF16>::E* d2colT;
    BotArgs a;
    int nsplit;
    float* part;
    static __device__ void run(const Gemm1Job& j, int v) {
        bwd_gemm1_body<BF16>(j.gp, j.code, j.d2colT, j.a, j.nsplit, j.part, v);
    }
};
template <bool BF16>
struct Gemm2Job {
    const void* gp;
    const uint8_t* code;
    const typename G2<BF16>::E* PT;
    BotArgs a;
    float* tt;
    static __device__ void run(const Gemm2Job& j, int v) { bwd_gemm2_body<BF16>(j.gp, j.code, j.PT, j.a, j.tt, v); }
};
struct Dd1ReduceJob {
    const float* part;
    BotArgs a;
    int nsplit;
    float* dd1;
    static __device__ void run(const Dd1ReduceJob& j, int v) { bwd_dd1_reduce_body<float>(j.part, j.a, j.nsplit, j.dd1, v); }
};
struct Col2imJob {
    const float* tt;
    BotArgs a;
    float* dd2;
    static __device__ void run(const Col2imJob& j, int v) { bwd_col2im_body(j.tt, j.a, j.dd2, v); }
};

BotArgs make_bot(const Geom& g) {
    BotArgs a;
    a.W1 = g.W1;
    a.H1 = g.H1;
    a.W2 = g.W2;
    a.H2 = g.H2;
    a.n0x = g.gx[0];
    a.natom = g.gx[0] * g.gy[0];
    a.h1 = g.h[1];
    a.w1 = g.w[1];
    a.Wp = (g.W2 + kPadW - 1) / kPadW * kPadW;
    a.H2p = (g.H2 + kPadH - 1) / kPadH * kPadH;
    a.Xp = a.Wp * a.H2p;
    a.Pp = (a.natom + G1<true>::M - 1) / G1<true>::M * G1<true>::M;
    a.pm = a.h1 * a.w1;
    return a;
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline unsigned g8(int nblocks) { return (unsigned)(((nblocks + 7) / 8) * 8); }

// Byte offsets of D2colT and PT inside the operand scratch region.
struct DenseLayout {
    size_t d2col, pt, total;
};
DenseLayout dense_layout(const BotArgs& a, size_t es) {
    DenseLayout d;
    d.d2col = 0;
    d.pt = align256((size_t)144 * a.Xp * es);
    d.total = d.pt + align256((size_t)144 * a.Pp * es);
    return d;
}

struct BotPlan {
    BotArgs a;
    int ns, d2_blocks, pt_blocks, g1_blocks, g2_blocks, red_blocks, c2i_blocks;
};

}  // namespace

int bwd_nsplit(const Geom& g) {
    // Enough blocks for the 256 CUs (patch tiles x K splits >= ~1024), but
    // at least 8192 target positions per split: small pairs then add few
    // partial sums, which matters when many of them share the GPU in a batch.
    // The count depends on the pair alone, so a batch sums in the same order
    // as the single-pair call.
    const BotArgs a = make_bot(g);
    const int ptiles = a.Pp / G1<true>::M;
    int ns = (1024 + ptiles - 1) / ptiles;
    if (ns > a.Xp / 8192) ns = a.Xp / 8192;
    if (ns > 64) ns = 64;
    if (ns > 8) ns &= ~7;   // whole groups of 8 splits
    if (ns < 1) ns = 1;
    return ns;
}

namespace {
BotPlan bot_plan(const Geom& g) {
    BotPlan b;
    b.a = make_bot(g);
    b.ns = bwd_nsplit(g);
    b.d2_blocks = (int)(((size_t)144 * (b.a.Xp / 8) + 255) / 256);
    b.pt_blocks = (int)(((size_t)144 * (b.a.Pp / 8) + 255) / 256);
    b.g1_blocks = (b.a.Pp / G1<true>::M) * b.ns;
    b.g2_blocks = (b.a.H2p / G2<true>::TR) * (b.a.Wp / G2<true>::TW);
    b.red_blocks = (int)(((size_t)b.a.H1 * b.a.W1 * 9 + 255) / 256);
    b.c2i_blocks = (int)(((size_t)b.a.H2 * b.a.W2 * 9 + 255) / 256);
    return b;
}
}  // namespace

size_t bwd_dense_bytes(const Geom& g, int precision) {
    return dense_layout(make_bot(g), precision == DM_BF16 ? 2 : 4).total;
}

size_t bwd_t_bytes(const Geom& g, int precision) {
    if (precision == DM_FP64) return (size_t)g.W2 * g.H2 * 144 * 8;
    return (size_t)144 * make_bot(g).Xp * 4;
}

// The six stages of the bottom backward of one pair as job records (bf16
// selects BF16 MFMA operands and a BF16 pooled gradient gp), in launch order.
std::vector<JobRec> bot_jobs(bool bf16, const float* gp, const uint8_t* code, const float* d1, const float* d2,
                             const Geom& g, float* part, float* tbuf, void* dense, float* dd1, float* dd2) {
    const BotPlan b = bot_plan(g);
    const DenseLayout d = dense_layout(b.a, bf16 ? 2 : 4);
    char* base = static_cast<char*>(dense);
    std::vector<JobRec> r(6);
    if (bf16) {
        uint16_t* dc = (uint16_t*)(base + d.d2col);
        uint16_t* pt = (uint16_t*)(base + d.pt);
        r[0].set(JK_D2COL_BF16, b.d2_blocks, 0, D2colJob<true>{d2, b.a, dc});
        r[1].set(JK_PATCH_BF16, b.pt_blocks, 0, PtJob<uint16_t>{d1, b.a, pt});
        r[2].set(JK_DD1_BF16, b.g1_blocks, 0, Gemm1Job<true>{gp, code, dc, b.a, b.ns, part});
        r[3].set(JK_TG_BF16, b.g2_blocks, 0, Gemm2Job<true>{gp, code, pt, b.a, tbuf});
    } else {
        float* dc = (float*)(base + d.d2col);
        float* pt = (float*)(base + d.pt);
        r[0].set(JK_D2COL_F32, b.d2_blocks, 0, D2colJob<false>{d2, b.a, dc});
        r[1].set(JK_PATCH_F32, b.pt_blocks, 0, PtJob<float>{d1, b.a, pt});
        r[2].set(JK_DD1_F32, b.g1_blocks, 0, Gemm1Job<false>{gp, code, dc, b.a, b.ns, part});
        r[3].set(JK_TG_F32, b.g2_blocks, 0, Gemm2Job<false>{gp, code, pt, b.a, tbuf});
    }
    r[4].set(JK_DD1_REDUCE, b.red_blocks, 0, Dd1ReduceJob{part, b.a, b.ns, dd1});
    r[5].set(JK_COL2IM, b.c2i_blocks, 0, Col2imJob{tbuf, b.a, dd2});
    return r;
}

hipError_t launch_group_bot(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_D2COL_BF16: return launch_grouped<D2colJob<true>, 256, 1>(gl, s);
        case JK_D2COL_F32: return launch_grouped<D2colJob<false>, 256, 1>(gl, s);
        case JK_PATCH_BF16: return launch_grouped<PtJob<uint16_t>, 256, 1>(gl, s);
        case JK_PATCH_F32: return launch_grouped<PtJob<float>, 256, 1>(gl, s);
        case JK_DD1_BF16: return launch_grouped<Gemm1Job<true>, 256, 2>(gl, s);
        case JK_DD1_F32: return launch_grouped<Gemm1Job<false>, 256, 2>(gl, s);
        case JK_TG_BF16: return launch_grouped<Gemm2Job<true>, 256, 2>(gl, s);
        case JK_TG_F32: return launch_grouped<Gemm2Job<false>, 256, 2>(gl, s);
        case JK_DD1_REDUCE: return launch_grouped<Dd1ReduceJob, 256, 1>(gl, s);
        case JK_COL2IM: return launch_grouped<Col2imJob, 256, 1>(gl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_bwd_bottom(int mode, const T* gp, const uint8_t* code, const T* d1, const T* d2, const Geom& g,
                             T* part, T* tbuf, void* dense, T* dd1, T* dd2, hipStream_t s) {
#define DM_SUB(name, ...)                  \
    do {                                   \
        timing_begin(name, 0, s);          \
        hipLaunchKernelGGL(__VA_ARGS__);   \
        timing_end(s);                     \
    } while (0)
    if (mode == 2) {  // reference kernels
        const BotArgs a = make_bot(g);
        const size_t n1 = (size_t)a.natom * 144, n2 = (size_t)a.H2 * a.W2 * 144;
        const size_t r1 = (size_t)a.H1 * a.W1 * 9, r2 = (size_t)a.H2 * a.W2 * 9;
        DM_SUB("bwd_dd1_ref", k_bwd_dd1_ref<T>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, gp, code, d2, a, part);
        DM_SUB("bwd_t_ref", k_bwd_t_ref<T>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, gp, code, d1, a, tbuf);
        DM_SUB("bwd_dd1_reduce", k_bwd_dd1_reduce<T>, dim3((unsigned)((r1 + 255) / 256)), dim3(256), 0, s, part, a, 1, dd1);
        DM_SUB("bwd_col2im", k_bwd_col2im_ref<T>, dim3((unsigned)((r2 + 255) / 256)), dim3(256), 0, s, tbuf, a, dd2);
        return hipGetLastError();
    }
    if constexpr (std::is_same<T, float>::value) {
        const BotPlan b = bot_plan(g);
        const BotArgs& a = b.a;
        const DenseLayout d = dense_layout(a, mode == 1 ? 2 : 4);
        char* base = static_cast<char*>(dense);
        if (mode == 1) {
            uint16_t* dc = (uint16_t*)(base + d.d2col);
            uint16_t* pt = (uint16_t*)(base + d.pt);
            DM_SUB("bwd_d2col", k_bwd_d2col<true>, dim3(b.d2_blocks), dim3(256), 0, s, d2, a, dc);
            DM_SUB("bwd_pt", k_bwd_pt<uint16_t>, dim3(b.pt_blocks), dim3(256), 0, s, d1, a, pt);
            DM_SUB("bwd_dd1_gemm", k_bwd_gemm1<true>, dim3(g8(b.g1_blocks)), dim3(256), 0, s, gp, code, dc, a, b.ns,
                   part, b.g1_blocks);
            DM_SUB("bwd_t_gemm", k_bwd_gemm2<true>, dim3(g8(b.g2_blocks)), dim3(256), 0, s, gp, code, pt, a, tbuf,
                   b.g2_blocks);
        } else {
            float* dc = (float*)(base + d.d2col);
            float* pt = (float*)(base + d.pt);
            DM_SUB("bwd_d2col", k_bwd_d2col<false>, dim3(b.d2_blocks), dim3(256), 0, s, d2, a, dc);
            DM_SUB("bwd_pt", k_bwd_pt<float>, dim3(b.pt_blocks), dim3(256), 0, s, d1, a, pt);
            DM_SUB("bwd_dd1_gemm", k_bwd_gemm1<false>, dim3(g8(b.g1_blocks)), dim3(256), 0, s, gp, code, dc, a, b.ns,
                   part, b.g1_blocks);
            DM_SUB("bwd_t_gemm", k_bwd_gemm2<false>, dim3(g8(b.g2_blocks)), dim3(256), 0, s, gp, code, pt, a, tbuf,
                   b.g2_blocks);
        }
        DM_SUB("bwd_dd1_reduce", k_bwd_dd1_reduce<float>, dim3(b.red_blocks), dim3(256), 0, s, part, a, b.ns, dd1);
        DM_SUB("bwd_col2im", k_bwd_col2im, dim3(b.c2i_blocks), dim3(256), 0, s, tbuf, a, dd2);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
#undef DM_SUB
}

template hipError_t launch_bwd_bottom<float>(int, const float*, const uint8_t*, const float*, const float*,
                                             const Geom&, float*, float*, void*, float*, float*, hipStream_t);
template hipError_t launch_bwd_bottom<double>(int, const double*, const uint8_t*, const double*, const double*,
                                              const Geom&, double*, double*, void*, double*, double*, hipStream_t);

}  // namespace dm
