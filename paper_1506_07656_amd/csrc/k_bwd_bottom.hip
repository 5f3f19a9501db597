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
// Matrix-core path (FP32 or BF16 operands, FP32 accumulation):
//  - dA_0 is written once, densely, by a gather over the <= 4 candidates in
//    a fixed order (deterministic), as a [Pp][Xp] array: target positions on
//    an H2p x Wp grid (width rounded up to 8, so rows of 8 values are
//    16-byte aligned, height up to 16, so Xp is a multiple of 128), patches padded to Pp
//    (a multiple of 128); padding entries are 0, so GEMM tiles never check
//    bounds.
//  - GEMM 1 (M = patches, N = 144, K = positions, split over K) and GEMM 2
//    (M = 144, N = positions, K = patches) read operands that are contiguous
//    along K: dA_0 rows, the transposed im2col of D2 ([144][Xp], built once)
//    and the transposed patch matrix of D1 ([144][Pp], built once).  GEMM 2
//    needs dA_0 along patches: 8 x 8 blocks are transposed in registers on
//    their way into LDS.  Tiles go through LDS with the next chunk's loads in
//    flight.  Split partial sums are added in a fixed order.
//
// Reference kernels (thread per output, direct loops) serve the FP64
// instantiation used by the finite-difference check.
#include <type_traits>

#include "dm_group.h"

namespace dm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
// Native 16-byte vector: copies are plain loads and stores, never memcpy of a
// struct, so arrays of them stay in registers.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct BotArgs {
    int W1, H1, W2, H2, n0x, natom, h1, w1;
    int Wp, H2p, Xp, Pp;   // padded dense layout (matrix-core path)
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

// ---------------------------------------------------------------- dense dA_0
// Block: one patch x 32 target rows x 256 target columns of the padded grid,
// accumulated in LDS.  Each pooled entry (ry, rx) sends its gradient to the
// one position its code names, (2 ry + my, 2 rx + mx); entries with the same
// parities of ry and rx never name the same position, so the four parity
// classes are added in four passes, in a fixed order, without atomics
// (deterministic).  Codes never name positions outside I' (the forward pool
// never selects one), so the padding of the grid stays 0.  A thread owns a
// 2 x 2 quad of pooled entries per round; then the tile leaves as rows of 8
// values (16 bytes in BF16).
constexpr int DA_ROWS = 32, DA_COLS = 256;
constexpr int DA_QR = DA_ROWS / 4 + 1, DA_QC = DA_COLS / 4 + 1;   // quads reaching the tile
constexpr int DA_NQ = DA_QR * DA_QC, DA_ROUNDS = (DA_NQ + 255) / 256;
constexpr int kOOB = 0x7ffffff0;                                   // buffer byte offset past any map

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

template <typename E>
__device__ __forceinline__ void bwd_da_body(const float* __restrict__ gp, const uint8_t* __restrict__ code, const BotArgs& a,
                                   int nct, E* __restrict__ dA, int bid) {
    __shared__ __align__(16) float sT[DA_ROWS][DA_COLS];
    const int tid = threadIdx.x;
    const int nband = (a.H2p + DA_ROWS - 1) / DA_ROWS;
    const int ct = bid % nct, rest = bid / nct, band = rest % nband, p = rest / nband;
    const int Y0 = band * DA_ROWS, X0 = ct * DA_COLS;
    const int ry0 = Y0 >> 1, rx0 = X0 >> 1;
    const uint32_t pm = (uint32_t)a.h1 * a.w1;
    const uint32_t nrec = __builtin_amdgcn_readfirstlane(p < a.natom ? pm : 0u);
    // BF16 operands come with a BF16 pooled gradient, FP32 with FP32
    constexpr bool G16 = std::is_same<E, uint16_t>::value;
    constexpr int gsz = G16 ? 2 : 4;   // bytes per stored gradient entry
    const auto rsG = buf_rsrc(reinterpret_cast<const char*>(gp) + (size_t)p * pm * gsz, nrec * gsz),
               rsM = buf_rsrc(code + (size_t)p * pm, nrec);
    // the quads' gradients and codes, in flight while the tile is cleared
    float g[DA_ROUNDS][4];
    int m[DA_ROUNDS][4];
#pragma unroll
    for (int k = 0; k < DA_ROUNDS; ++k) {
        const int q = tid + 256 * k, qi = q / DA_QC, qj = q - qi * DA_QC;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ry = ry0 + 2 * qi + (e >> 1), rx = rx0 + 2 * qj + (e & 1);
            const bool ok = q < DA_NQ && rx < a.w1 && ry < a.h1;
            const int off = ry * a.w1 + rx;   // used only when ok
            if constexpr (G16)
                g[k][e] = __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rsG, ok ? off * 2 : kOOB, 0, 0)
                                          << 16);
            else
                g[k][e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsG, ok ? off * 4 : kOOB, 0, 0));
            m[k][e] = __builtin_amdgcn_raw_buffer_load_b8(rsM, ok ? off : kOOB, 0, 0);
        }
    }
    for (int e = tid; e < DA_ROWS * DA_COLS / 4; e += 256) reinterpret_cast<float4*>(&sT[0][0])[e] = float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 4; ++e) {   // parity class (ry - ry0) & 1 = e >> 1, (rx - rx0) & 1 = e & 1
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DA_ROUNDS; ++k) {
            const int q = tid + 256 * k, qi = q / DA_QC, qj = q - qi * DA_QC;
            const int my = (m[k][e] * 11) >> 5, mx = m[k][e] - 3 * my;   // code = 3 (my + 1) + (mx + 1), 0..8
            const int ly = 4 * qi + 2 * (e >> 1) + my - 1, lx = 4 * qj + 2 * (e & 1) + mx - 1;
            // no two entries of one class meet: an LDS add without return is exactly old + g
            if (g[k][e] != 0.f && ly >= 0 && ly < DA_ROWS && lx >= 0 && lx < DA_COLS) atomicAdd(&sT[ly][lx], g[k][e]);
        }
    }
    __syncthreads();
    const int grp = tid & 31, xb = X0 + 8 * grp;
    if (xb >= a.Wp) return;
#pragma unroll
    for (int k = 0; k < DA_ROWS / 8; ++k) {
        const int row = (tid >> 5) + 8 * k, y = Y0 + row;
        if (y >= a.H2p) break;
        const float4 v0 = *reinterpret_cast<const float4*>(&sT[row][8 * grp]);
        const float4 v1 = *reinterpret_cast<const float4*>(&sT[row][8 * grp + 4]);
        const float out[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        store8<E>(dA + (size_t)p * a.Xp + (size_t)y * a.Wp + xb, out);
    }
}

// Transposed im2col of D2: D2colT[k][x] = D2[x + d_k][c_k] on the padded grid.
template <typename E>
__device__ inline void bwd_d2col_body(const float* __restrict__ d2, const BotArgs& a, E* __restrict__ d2colT,
                                      int bid) {
    const size_t v = (size_t)bid * 256 + threadIdx.x;   // one group of 8 positions
    const int gpr = a.Xp / 8;
    if (v >= (size_t)144 * gpr) return;
    const int k = v / gpr, x0 = (int)(v - (size_t)k * gpr) * 8;
    const int y = x0 / a.Wp, xx0 = x0 - y * a.Wp;
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = (y < a.H2 && xx0 + q < a.W2) ? d2_at(d2, a, y, xx0 + q, k) : 0.f;
    store8<E>(d2colT + (size_t)k * a.Xp + x0, out);
}

// Transposed patch matrix of D1: PT[k][p] = D1[p + d_k][c_k] (0 for padding patches).
template <typename E>
__device__ inline void bwd_pt_body(const float* __restrict__ d1, const BotArgs& a, E* __restrict__ PT, int bid) {
    const size_t v = (size_t)bid * 256 + threadIdx.x;
    const int gpr = a.Pp / 8;
    if (v >= (size_t)144 * gpr) return;
    const int k = v / gpr, p0 = (int)(v - (size_t)k * gpr) * 8;
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] = p0 + q < a.natom ? d1_at(d1, a, p0 + q, k) : 0.f;
    store8<E>(PT + (size_t)k * a.Pp + p0, out);
}

// ---------------------------------------------------------------- GEMMs
constexpr int GK = 64;     // K chunk
constexpr int G1M = 128;   // GEMM 1: patches per block
constexpr int G2N = 128;   // GEMM 2: positions per block

template <bool BF16>
struct Op {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    static constexpr int VPR = BF16 ? 8 : 4;     // values per 16-byte vector
    static constexpr int PAD = BF16 ? 8 : 4;     // LDS row padding (keeps rows 16-byte aligned)
    static constexpr int CV = GK / VPR;          // vectors per chunk row
};

// C[M=128 patches][N=144] += A[M][K] * B[N][K]^T over the chunks of one split.
template <bool BF16>
__device__ __forceinline__ void bwd_gemm1_body(const typename Op<BF16>::E* __restrict__ dA,
                                      const typename Op<BF16>::E* __restrict__ d2colT, const BotArgs& a, int nsplit,
                                      float* __restrict__ part, int bid) {
    typedef Op<BF16> O;
    typedef typename O::E E;
    __shared__ __align__(16) E sA[G1M][GK + O::PAD];
    __shared__ __align__(16) E sB[144][GK + O::PAD];
    constexpr int NA = G1M * O::CV / 256, NB = (144 * O::CV + 255) / 256;
    const int ptiles = a.Pp / G1M;
    const int split = bid / ptiles, ptile = bid - split * ptiles;
    const int kper = ((a.Xp / GK + nsplit - 1) / nsplit) * GK;
    const int k_begin = split * kper, k_end = min(a.Xp, k_begin + kper);
    const int P0 = ptile * G1M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    // Prefetch registers, filled by unconditional loads (rows of the B chunk
    // past its 144 are clamped and not stored): they must stay in VGPRs.
    u32x4 ra[NA], rb[NB];
    size_t aoff[NA], boff[NB];   // element offsets of each vector's row at chunk start 0
    int aidx[NA], bidx[NB];   // LDS destinations (element index), -1 = none
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int v = tid + 256 * i, r = v / O::CV, c = v - r * O::CV;
        aoff[i] = (size_t)(P0 + r) * a.Xp + c * O::VPR;
        aidx[i] = r * (GK + O::PAD) + c * O::VPR;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int v = tid + 256 * i, vc = min(v, 144 * O::CV - 1), r = vc / O::CV, c = vc - r * O::CV;
        boff[i] = (size_t)r * a.Xp + c * O::VPR;
        bidx[i] = v < 144 * O::CV ? r * (GK + O::PAD) + c * O::VPR : -1;
    }
    f4 acc[2][9];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    if (k_begin < k_end) {
#pragma unroll
        for (int i = 0; i < NA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(dA + aoff[i] + k_begin);
#pragma unroll
        for (int i = 0; i < NB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(d2colT + boff[i] + k_begin);
    }
    for (int k0 = k_begin; k0 < k_end; k0 += GK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i) *reinterpret_cast<u32x4*>(&sA[0][0] + aidx[i]) = ra[i];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (bidx[i] >= 0) *reinterpret_cast<u32x4*>(&sB[0][0] + bidx[i]) = rb[i];
        __syncthreads();
        if (k0 + GK < k_end) {   // next chunk in flight during the MFMAs
#pragma unroll
            for (int i = 0; i < NA; ++i) ra[i] = *reinterpret_cast<const u32x4*>(dA + aoff[i] + k0 + GK);
#pragma unroll
            for (int i = 0; i < NB; ++i) rb[i] = *reinterpret_cast<const u32x4*>(d2colT + boff[i] + k0 + GK);
        }
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < GK / 32; ++s) {
                bf8 av[2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) av[mt] = as_bf8(&sA[wave * 32 + mt * 16 + n][32 * s + 8 * g]);
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const bf8 bv = as_bf8(&sB[16 * nt + n][32 * s + 8 * g]);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv, acc[mt][nt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 4
            for (int t = 0; t < GK / 4; ++t) {
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

// T[M=144][N=128 positions] += PT[M][K] * dA[K][N] over all patch chunks.
// The dA chunk (64 patches x 128 positions) comes through registers, its
// 8 x 8 (BF16) or 4 x 4 (FP32) blocks transposed so that LDS holds it as
// [position][patch]; the PT chunk is copied as it is.
template <bool BF16>
__device__ __forceinline__ void bwd_gemm2_body(const typename Op<BF16>::E* __restrict__ dA,
                                      const typename Op<BF16>::E* __restrict__ PT, const BotArgs& a,
                                      float* __restrict__ tt, int bid) {
    typedef Op<BF16> O;
    typedef typename O::E E;
    __shared__ __align__(16) E sA[144][GK + O::PAD];   // PT chunk [k][patch]
    __shared__ __align__(16) E sB[G2N][GK + O::PAD];   // dA chunk [position][patch]
    const int X0 = bid * G2N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    // BF16: threads 0..127 take one 8x8 dA block each, threads 128..255 the
    // PT chunk; FP32: every thread takes two 4x4 dA blocks and part of PT.
    constexpr int BR = BF16 ? 8 : 4, NBLK = BF16 ? 1 : 2;
    constexpr int NTH_A = BF16 ? 128 : 256, NTH_P = BF16 ? 128 : 256;   // threads per role
    constexpr int NPT = (144 * O::CV + NTH_P - 1) / NTH_P;             // PT vectors per thread
    // Prefetch registers, filled by unconditional loads (PT rows past 144 are
    // clamped and not stored) so that they stay in VGPRs.
    u32x4 rd[NBLK][BR];
    u32x4 rp[NPT];
    const bool loader_a = BF16 ? tid < 128 : true;    // wave-uniform
    const bool loader_p = BF16 ? tid >= 128 : true;
    const int tp = BF16 ? tid - 128 : tid;
    const E* dsrc[NBLK];   // first dA row of this thread's block at chunk start 0
    int dcol[NBLK], drow[NBLK];
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
        // patch block fastest: each LDS row gets contiguous stores
        const int blk = (loader_a ? tid : 0) + NTH_A * b;
        const int pbn = GK / BR, xb = blk / pbn, pb = blk - xb * pbn;
        dsrc[b] = dA + (size_t)(BR * pb) * a.Xp + X0 + BR * xb;
        drow[b] = BR * xb;
        dcol[b] = BR * pb;
    }
    const E* psrc[NPT];
    int pidx[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int v = (loader_p ? tp : 0) + NTH_P * i, vc = min(v, 144 * O::CV - 1), r = vc / O::CV,
                  c = vc - r * O::CV;
        psrc[i] = PT + (size_t)r * a.Pp + c * O::VPR;
        pidx[i] = v < 144 * O::CV ? r * (GK + O::PAD) + c * O::VPR : -1;
    }
    f4 acc[9][2];
#pragma unroll
    for (int mt = 0; mt < 9; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
#define DM_G2_LOAD(P0_)                                                                              \
    do {                                                                                             \
        if (loader_a) {                                                                              \
            _Pragma("unroll") for (int b = 0; b < NBLK; ++b)                                         \
                _Pragma("unroll") for (int i = 0; i < BR; ++i) rd[b][i] =                            \
                    *reinterpret_cast<const u32x4*>(dsrc[b] + (size_t)((P0_) + i) * a.Xp);           \
        }                                                                                            \
        if (loader_p) {                                                                              \
            _Pragma("unroll") for (int i = 0; i < NPT; ++i) rp[i] =                                  \
                *reinterpret_cast<const u32x4*>(psrc[i] + (P0_));                                    \
        }                                                                                            \
    } while (0)
    DM_G2_LOAD(0);
    for (int p0 = 0; p0 < a.Pp; p0 += GK) {
        __syncthreads();
        if (loader_a) {
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                if constexpr (BF16) {
                    // rd[b][i] = 8 bf16 of patch row i (positions 2j, 2j+1 in dword j);
                    // column q (position) = 8 patches, packed 2 per dword.
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        u32x4 o;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t lo = rd[b][2 * j][q >> 1], hi = rd[b][2 * j + 1][q >> 1];
                            o[j] = (q & 1) ? ((lo >> 16) | (hi & 0xFFFF0000u)) : ((lo & 0xFFFFu) | (hi << 16));
                        }
                        *reinterpret_cast<u32x4*>(&sB[drow[b] + q][dcol[b]]) = o;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<u32x4*>(&sB[drow[b] + q][dcol[b]]) =
                            u32x4{rd[b][0][q], rd[b][1][q], rd[b][2][q], rd[b][3][q]};
                }
            }
        }
        if (loader_p) {
#pragma unroll
            for (int i = 0; i < NPT; ++i)
                if (pidx[i] >= 0) *reinterpret_cast<u32x4*>(&sA[0][0] + pidx[i]) = rp[i];
        }
        __syncthreads();
        if (p0 + GK < a.Pp) DM_G2_LOAD(p0 + GK);
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < GK / 32; ++s) {
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
            for (int t = 0; t < GK / 4; ++t) {
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
#pragma unroll
    for (int mt = 0; mt < 9; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                tt[(size_t)(16 * mt + 4 * g + j) * a.Xp + X0 + wave * 32 + nt * 16 + n] = acc[mt][nt][j];
}
#undef DM_G2_LOAD

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
// works through one contiguous range (GEMM 1: the patch tiles of one K split
// share its slice of the im2col operand in that XCD's L2).
__device__ inline int xcd_block(int nblocks) {
    const int per = (nblocks + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <typename E>
__global__ __launch_bounds__(256) void k_bwd_da(const float* __restrict__ gp, const uint8_t* __restrict__ code,
                                                BotArgs a, int nct, E* __restrict__ dA, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid < nblocks) bwd_da_body<E>(gp, code, a, nct, dA, bid);
}
template <typename E>
__global__ __launch_bounds__(256) void k_bwd_d2col(const float* __restrict__ d2, BotArgs a, E* __restrict__ d2colT) {
    bwd_d2col_body<E>(d2, a, d2colT, blockIdx.x);
}
template <typename E>
__global__ __launch_bounds__(256) void k_bwd_pt(const float* __restrict__ d1, BotArgs a, E* __restrict__ PT) {
    bwd_pt_body<E>(d1, a, PT, blockIdx.x);
}
template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_gemm1(const typename Op<BF16>::E* __restrict__ dA,
                                                   const typename Op<BF16>::E* __restrict__ d2colT, BotArgs a,
                                                   int nsplit, float* __restrict__ part, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid < nblocks) bwd_gemm1_body<BF16>(dA, d2colT, a, nsplit, part, bid);
}
template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_gemm2(const typename Op<BF16>::E* __restrict__ dA,
                                                   const typename Op<BF16>::E* __restrict__ PT, BotArgs a,
                                                   float* __restrict__ tt, int nblocks) {
    const int bid = xcd_block(nblocks);
    if (bid < nblocks) bwd_gemm2_body<BF16>(dA, PT, a, tt, bid);
}
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_dd1_reduce(const T* __restrict__ part, BotArgs a, int nsplit,
                                                        T* __restrict__ dd1) {
    bwd_dd1_reduce_body<T>(part, a, nsplit, dd1, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_bwd_col2im(const float* __restrict__ tt, BotArgs a, float* __restrict__ dd2) {
    bwd_col2im_body(tt, a, dd2, blockIdx.x);
}

template <typename E>
struct DaJob {
    const float* gp;
    const uint8_t* code;
    BotArgs a;
    int nct;
    E* dA;
    static __device__ void run(const DaJob& j, int v) { bwd_da_body<E>(j.gp, j.code, j.a, j.nct, j.dA, v); }
};
template <typename E>
struct D2colJob {
    const float* d2;
    BotArgs a;
    E* d2colT;
    static __device__ void run(const D2colJob& j, int v) { bwd_d2col_body<E>(j.d2, j.a, j.d2colT, v); }
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
    const typename Op<BF16>::E *dA, *d2colT;
    BotArgs a;
    int nsplit;
    float* part;
    static __device__ void run(const Gemm1Job& j, int v) { bwd_gemm1_body<BF16>(j.dA, j.d2colT, j.a, j.nsplit, j.part, v); }
};
template <bool BF16>
struct Gemm2Job {
    const typename Op<BF16>::E *dA, *PT;
    BotArgs a;
    float* tt;
    static __device__ void run(const Gemm2Job& j, int v) { bwd_gemm2_body<BF16>(j.dA, j.PT, j.a, j.tt, v); }
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
    a.Wp = (g.W2 + 7) & ~7;
    a.H2p = (g.H2 + 15) & ~15;
    a.Xp = a.Wp * a.H2p;
    a.Pp = (a.natom + G1M - 1) / G1M * G1M;
    return a;
}

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline unsigned g8(int nblocks) { return (unsigned)(((nblocks + 7) / 8) * 8); }

// Byte offsets of dA_0, D2colT and PT inside the dense scratch region.
struct DenseLayout {
    size_t da, d2col, pt, total;
};
DenseLayout dense_layout(const BotArgs& a, size_t es) {
    DenseLayout d;
    d.da = 0;
    d.d2col = align256((size_t)a.Pp * a.Xp * es);
    d.pt = d.d2col + align256((size_t)144 * a.Xp * es);
    d.total = d.pt + align256((size_t)144 * a.Pp * es);
    return d;
}

struct BotPlan {
    BotArgs a;
    int ns, nct, da_blocks, d2_blocks, pt_blocks, g1_blocks, g2_blocks, red_blocks, c2i_blocks;
};

}  // namespace

int bwd_nsplit(const Geom& g) {
    // Enough blocks for the 256 CUs (patch tiles x K splits >= ~1024), but
    // at least 8192 target positions per split: small pairs then add few
    // partial sums, which matters when many of them share the GPU in a batch.
    // The count depends on the pair alone, so a batch sums in the same order
    // as the single-pair call.
    const int natom = g.gx[0] * g.gy[0];
    const int ptiles = (natom + G1M - 1) / G1M;
    const int xp = ((g.W2 + 7) & ~7) * ((g.H2 + 15) & ~15);
    int ns = (1024 + ptiles - 1) / ptiles;
    if (ns > xp / 8192) ns = xp / 8192;
    if (ns > 64) ns = 64;
    if (ns < 1) ns = 1;
    return ns;
}

namespace {
BotPlan bot_plan(const Geom& g) {
    BotPlan b;
    b.a = make_bot(g);
    b.ns = bwd_nsplit(g);
    b.nct = (b.a.Wp + DA_COLS - 1) / DA_COLS;
    b.da_blocks = b.a.Pp * ((b.a.H2p + DA_ROWS - 1) / DA_ROWS) * b.nct;
    b.d2_blocks = (int)(((size_t)144 * (b.a.Xp / 8) + 255) / 256);
    b.pt_blocks = (int)(((size_t)144 * (b.a.Pp / 8) + 255) / 256);
    b.g1_blocks = (b.a.Pp / G1M) * b.ns;
    b.g2_blocks = b.a.Xp / G2N;
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

// The seven stages of the bottom backward of one pair as job records (FP32
// storage; bf16 selects BF16 MFMA operands), in launch order.
std::vector<JobRec> bot_jobs(bool bf16, const float* gp, const uint8_t* code, const float* d1, const float* d2,
                             const Geom& g, float* part, float* tbuf, void* dense, float* dd1, float* dd2) {
    const BotPlan b = bot_plan(g);
    const DenseLayout d = dense_layout(b.a, bf16 ? 2 : 4);
    char* base = static_cast<char*>(dense);
    std::vector<JobRec> r(7);
    if (bf16) {
        uint16_t* dA = (uint16_t*)(base + d.da);
        uint16_t* dc = (uint16_t*)(base + d.d2col);
        uint16_t* pt = (uint16_t*)(base + d.pt);
        r[0].set(JK_BWD_DA_BF16, b.da_blocks, 0, DaJob<uint16_t>{gp, code, b.a, b.nct, dA});
        r[1].set(JK_D2COL_BF16, b.d2_blocks, 0, D2colJob<uint16_t>{d2, b.a, dc});
        r[2].set(JK_PATCH_BF16, b.pt_blocks, 0, PtJob<uint16_t>{d1, b.a, pt});
        r[3].set(JK_DD1_BF16, b.g1_blocks, 0, Gemm1Job<true>{dA, dc, b.a, b.ns, part});
        r[4].set(JK_TG_BF16, b.g2_blocks, 0, Gemm2Job<true>{dA, pt, b.a, tbuf});
    } else {
        float* dA = (float*)(base + d.da);
        float* dc = (float*)(base + d.d2col);
        float* pt = (float*)(base + d.pt);
        r[0].set(JK_BWD_DA_F32, b.da_blocks, 0, DaJob<float>{gp, code, b.a, b.nct, dA});
        r[1].set(JK_D2COL_F32, b.d2_blocks, 0, D2colJob<float>{d2, b.a, dc});
        r[2].set(JK_PATCH_F32, b.pt_blocks, 0, PtJob<float>{d1, b.a, pt});
        r[3].set(JK_DD1_F32, b.g1_blocks, 0, Gemm1Job<false>{dA, dc, b.a, b.ns, part});
        r[4].set(JK_TG_F32, b.g2_blocks, 0, Gemm2Job<false>{dA, pt, b.a, tbuf});
    }
    r[5].set(JK_DD1_REDUCE, b.red_blocks, 0, Dd1ReduceJob{part, b.a, b.ns, dd1});
    r[6].set(JK_COL2IM, b.c2i_blocks, 0, Col2imJob{tbuf, b.a, dd2});
    return r;
}

hipError_t launch_group_bot(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_BWD_DA_BF16: return launch_grouped<DaJob<uint16_t>, 256, 1>(gl, s);
        case JK_BWD_DA_F32: return launch_grouped<DaJob<float>, 256, 1>(gl, s);
        case JK_D2COL_BF16: return launch_grouped<D2colJob<uint16_t>, 256, 1>(gl, s);
        case JK_D2COL_F32: return launch_grouped<D2colJob<float>, 256, 1>(gl, s);
        case JK_PATCH_BF16: return launch_grouped<PtJob<uint16_t>, 256, 1>(gl, s);
        case JK_PATCH_F32: return launch_grouped<PtJob<float>, 256, 1>(gl, s);
        case JK_DD1_BF16: return launch_grouped<Gemm1Job<true>, 256, 1>(gl, s);
        case JK_DD1_F32: return launch_grouped<Gemm1Job<false>, 256, 1>(gl, s);
        case JK_TG_BF16: return launch_grouped<Gemm2Job<true>, 256, 1>(gl, s);
        case JK_TG_F32: return launch_grouped<Gemm2Job<false>, 256, 1>(gl, s);
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
            uint16_t* dA = (uint16_t*)(base + d.da);
            uint16_t* dc = (uint16_t*)(base + d.d2col);
            uint16_t* pt = (uint16_t*)(base + d.pt);
            DM_SUB("bwd_da", k_bwd_da<uint16_t>, dim3(g8(b.da_blocks)), dim3(256), 0, s, gp, code, a, b.nct, dA,
                   b.da_blocks);
            DM_SUB("bwd_d2col", k_bwd_d2col<uint16_t>, dim3(b.d2_blocks), dim3(256), 0, s, d2, a, dc);
            DM_SUB("bwd_pt", k_bwd_pt<uint16_t>, dim3(b.pt_blocks), dim3(256), 0, s, d1, a, pt);
            DM_SUB("bwd_dd1_gemm", k_bwd_gemm1<true>, dim3(g8(b.g1_blocks)), dim3(256), 0, s, dA, dc, a, b.ns, part,
                   b.g1_blocks);
            DM_SUB("bwd_t_gemm", k_bwd_gemm2<true>, dim3(g8(b.g2_blocks)), dim3(256), 0, s, dA, pt, a, tbuf,
                   b.g2_blocks);
        } else {
            float* dA = (float*)(base + d.da);
            float* dc = (float*)(base + d.d2col);
            float* pt = (float*)(base + d.pt);
            DM_SUB("bwd_da", k_bwd_da<float>, dim3(g8(b.da_blocks)), dim3(256), 0, s, gp, code, a, b.nct, dA,
                   b.da_blocks);
            DM_SUB("bwd_d2col", k_bwd_d2col<float>, dim3(b.d2_blocks), dim3(256), 0, s, d2, a, dc);
            DM_SUB("bwd_pt", k_bwd_pt<float>, dim3(b.pt_blocks), dim3(256), 0, s, d1, a, pt);
            DM_SUB("bwd_dd1_gemm", k_bwd_gemm1<false>, dim3(g8(b.g1_blocks)), dim3(256), 0, s, dA, dc, a, b.ns, part,
                   b.g1_blocks);
            DM_SUB("bwd_t_gemm", k_bwd_gemm2<false>, dim3(g8(b.g2_blocks)), dim3(256), 0, s, dA, pt, a, tbuf,
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
