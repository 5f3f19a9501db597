// Adjoint of the bottom correlation (Eq. (3)) for the gradient pass.
//
// With g'_0(p, r) the gradient routed to pooled entry r of atomic patch p
// (see k_backward.hip), the gradient with respect to A_0 is
//   dA_0(p, x) = sum_{r: 2r + m_0(p, r) = x} g'_0(p, r)        (<= 4 candidates)
// and, with K index k = (dy, dx, c) over the 4x4 patch and 9 channels,
//   dD1[p + d_k][c_k] = 1/16 sum_x dA_0(p, x) D2[x + d_k][c_k]          (GEMM 1)
//   T[x][k]           =      sum_p dA_0(p, x) D1[p + d_k][c_k]          (GEMM 2)
//   dD2[y][c]         = 1/16 sum_{dy,dx} T[y - d][(d, c)]               (col2im)
// Atomic patches do not overlap, so GEMM 1 writes each D1 pixel once.  dA_0
// is rebuilt once from g'_0 and the argmax codes into a dense scratch array
// (BF16 or FP32, the GEMM operand type), which both GEMMs stream through LDS
// tiles on the matrix cores; partial sums over row splits are added in a
// fixed order, so the result is deterministic.
//
// Reference kernels (thread per output, direct loops) serve the FP64
// instantiation used by the finite-difference check.
#include <type_traits>

#include "dm_group.h"

namespace dm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct BotArgs {
    int W1, H1, W2, H2, n0x, natom, h1, w1;
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

// ---------------------------------------------------------------- dense dA_0
// dA_0 is written once, densely ([patch][target pixel], operand type E), and
// both contractions stream it with coalesced loads.
template <typename E>
__device__ inline void bwd_da_body(const float* __restrict__ gp, const uint8_t* __restrict__ code, const BotArgs& a,
                                   int xblocks, E* __restrict__ dA, int bid) {
    const int p = bid / xblocks, xb = bid - p * xblocks;
    const int npos = a.H2 * a.W2;
    const size_t pm = (size_t)a.h1 * a.w1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int x = xb * 1024 + u * 256 + threadIdx.x;
        if (x >= npos) continue;
        const int xy = x / a.W2, xx = x - xy * a.W2;
        const float v = dA_at(gp + p * pm, code + p * pm, a.h1, a.w1, xy, xx);
        if constexpr (std::is_same<E, float>::value) dA[(size_t)p * npos + x] = v;
        else dA[(size_t)p * npos + x] = to_bf16(v);
    }
}

// Patch matrix P[p][k] = D1[p + d_k][c_k] (k = (dy, dx, c)), operand type E.
template <typename E>
__device__ inline void bwd_patchmat_body(const float* __restrict__ d1, const BotArgs& a, E* __restrict__ P, int bid) {
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i >= (size_t)a.natom * 144) return;
    const int p = i / 144, k = i % 144;
    const float v = d1_at(d1, a, p, k);
    if constexpr (std::is_same<E, float>::value) P[i] = v;
    else P[i] = to_bf16(v);
}

// ---------------------------------------------------------------- GEMM 1: dD1
// Block: 128 patches (32 per wave = 2 M-tiles) x all 144 K columns (9
// N-tiles), reducing over the target rows of one split in chunks of 64
// pixels of one row: the dA tile [128][64] comes straight from the dense dA,
// the im2col tile [144][64] is built from an LDS copy of the 4 x 67 target
// pixels it covers.
constexpr int G1P = 128, KC = 64;

template <bool BF16>
__device__ inline void bwd_dd1_gemm_body(const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ dA,
                                         const float* __restrict__ d2, const BotArgs& a, int nsplit,
                                         float* __restrict__ part, int bid) {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    constexpr int PAD = BF16 ? 8 : 1;
    __shared__ __align__(16) E sA[G1P][KC + PAD];
    __shared__ __align__(16) E sB[144][KC + PAD];
    __shared__ float sD2[4][KC + 3][9];
    const int ptile = bid / nsplit, split = bid % nsplit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    const int npos = a.H2 * a.W2;
    const int rows_per = (a.H2 + nsplit - 1) / nsplit;
    const int y_begin = split * rows_per, y_end = min(a.H2, y_begin + rows_per);
    f4 acc[2][9];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int y = y_begin; y < y_end; ++y) {
        for (int x0 = 0; x0 < a.W2; x0 += KC) {
            __syncthreads();
            // target pixels rows y-2..y+1, columns x0-2..x0+KC, zero outside
            for (int e = tid; e < 4 * (KC + 3) * 9; e += 256) {
                const int r = e / ((KC + 3) * 9), rem = e - r * ((KC + 3) * 9);
                const int col = rem / 9, c = rem - col * 9;
                const int yy = y - 2 + r, xx = x0 - 2 + col;
                sD2[r][col][c] = (yy >= 0 && yy < a.H2 && xx >= 0 && xx < a.W2) ? d2[((size_t)yy * a.W2 + xx) * 9 + c] : 0.f;
            }
            for (int e = tid; e < G1P * KC; e += 256) {
                const int pl = e / KC, xi = e - pl * KC;
                const int p = ptile * G1P + pl, x = x0 + xi;
                E v = E(0);
                if (p < a.natom && x < a.W2) v = dA[(size_t)p * npos + y * a.W2 + x];
                sA[pl][xi] = v;
            }
            __syncthreads();
            for (int e = tid; e < 144 * KC; e += 256) {
                const int k = e / KC, xi = e - k * KC;
                const int dy = k / 36, dx = (k / 9) % 4, c = k % 9;
                const float v = (x0 + xi < a.W2) ? sD2[dy][xi + dx][c] : 0.f;
                if constexpr (BF16) sB[k][xi] = to_bf16(v); else sB[k][xi] = v;
            }
            __syncthreads();
            if constexpr (BF16) {
#pragma unroll
                for (int s = 0; s < KC / 32; ++s) {
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
#pragma unroll 2
                for (int t = 0; t < KC / 4; ++t) {
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
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = ptile * G1P + wave * 32 + mt * 16 + 4 * g + j;
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

// ---------------------------------------------------------------- GEMM 2: T
// Block: 128 target pixels (32 per wave = 2 M-tiles) x 144 columns, reducing
// over all patches in chunks of 64: dA tile kept transposed [pixel][patch]
// and patch tile [144][patch] in LDS.
template <bool BF16>
__device__ inline void bwd_t_gemm_body(const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ dA,
                                       const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ P,
                                       const BotArgs& a, float* __restrict__ tbuf, int bid) {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    constexpr int PAD = BF16 ? 8 : 1;
    __shared__ __align__(16) E sAT[128][64 + PAD];   // [pixel][patch]
    __shared__ __align__(16) E sP[144][64 + PAD];    // [k][patch]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    const int npos = a.H2 * a.W2;
    const int xb = bid * 128;
    f4 acc[2][9];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 9; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < a.natom; p0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * 128; e += 256) {
            const int pl = e / 128, xi = e - pl * 128;
            const int p = p0 + pl, x = xb + xi;
            sAT[xi][pl] = (p < a.natom && x < npos) ? dA[(size_t)p * npos + x] : E(0);
        }
        for (int e = tid; e < 64 * 144; e += 256) {
            const int pl = e / 144, k = e - pl * 144;
            const int p = p0 + pl;
            sP[k][pl] = p < a.natom ? P[(size_t)p * 144 + k] : E(0);
        }
        __syncthreads();
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                bf8 av[2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) av[mt] = as_bf8(&sAT[wave * 32 + mt * 16 + n][32 * s + 8 * g]);
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const bf8 bv = as_bf8(&sP[16 * nt + n][32 * s + 8 * g]);
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv, acc[mt][nt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 2
            for (int t = 0; t < 16; ++t) {
                const float a0 = sAT[wave * 32 + n][4 * t + g], a1 = sAT[wave * 32 + 16 + n][4 * t + g];
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const float bv = sP[16 * nt + n][4 * t + g];
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
                const int x = xb + wave * 32 + mt * 16 + 4 * g + j;
                if (x < npos) tbuf[(size_t)x * 144 + 16 * nt + n] = acc[mt][nt][j];
            }
}

// dD2[y][c] = 1/16 sum_d T[y - d][(d, c)]  (T is zero outside the target).
template <typename T>
__device__ inline void bwd_col2im_body(const T* __restrict__ tbuf, const BotArgs& a, T* __restrict__ dd2, int bid) {
    const size_t n = (size_t)a.H2 * a.W2 * 9;
    const size_t i = (size_t)bid * 256 + threadIdx.x;
    if (i >= n) return;
    const int c = i % 9;
    const int x = (i / 9) % a.W2, y = i / (9 * (size_t)a.W2);
    T v = 0;
    for (int dy = 0; dy < 4; ++dy) {
        const int qy = y + 2 - dy;          // position whose patch covers y at row offset dy
        if (qy < 0 || qy >= a.H2) continue;
        for (int dx = 0; dx < 4; ++dx) {
            const int qx = x + 2 - dx;
            if (qx < 0 || qx >= a.W2) continue;
            v += tbuf[((size_t)qy * a.W2 + qx) * 144 + dy * 36 + dx * 9 + c];
        }
    }
    dd2[i] = v / T(16);
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

template <typename E>
__global__ __launch_bounds__(256) void k_bwd_da(const float* __restrict__ gp, const uint8_t* __restrict__ code,
                                                BotArgs a, int xblocks, E* __restrict__ dA) {
    bwd_da_body<E>(gp, code, a, xblocks, dA, blockIdx.x);
}
template <typename E>
__global__ __launch_bounds__(256) void k_bwd_patchmat(const float* __restrict__ d1, BotArgs a, E* __restrict__ P) {
    bwd_patchmat_body<E>(d1, a, P, blockIdx.x);
}
template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_dd1_gemm(
    const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ dA, const float* __restrict__ d2,
    BotArgs a, int nsplit, float* __restrict__ part) {
    bwd_dd1_gemm_body<BF16>(dA, d2, a, nsplit, part, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_dd1_reduce(const T* __restrict__ part, BotArgs a, int nsplit,
                                                        T* __restrict__ dd1) {
    bwd_dd1_reduce_body<T>(part, a, nsplit, dd1, blockIdx.x);
}
template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_t_gemm(
    const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ dA,
    const typename std::conditional<BF16, uint16_t, float>::type* __restrict__ P, BotArgs a,
    float* __restrict__ tbuf) {
    bwd_t_gemm_body<BF16>(dA, P, a, tbuf, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_col2im(const T* __restrict__ tbuf, BotArgs a, T* __restrict__ dd2) {
    bwd_col2im_body<T>(tbuf, a, dd2, blockIdx.x);
}

template <typename E>
struct DaJob {
    const float* gp;
    const uint8_t* code;
    BotArgs a;
    int xblocks;
    E* dA;
    static __device__ void run(const DaJob& j, int v) { bwd_da_body<E>(j.gp, j.code, j.a, j.xblocks, j.dA, v); }
};
template <typename E>
struct PatchJob {
    const float* d1;
    BotArgs a;
    E* P;
    static __device__ void run(const PatchJob& j, int v) { bwd_patchmat_body<E>(j.d1, j.a, j.P, v); }
};
template <bool BF16>
struct Dd1Job {
    const typename std::conditional<BF16, uint16_t, float>::type* dA;
    const float* d2;
    BotArgs a;
    int nsplit;
    float* part;
    static __device__ void run(const Dd1Job& j, int v) { bwd_dd1_gemm_body<BF16>(j.dA, j.d2, j.a, j.nsplit, j.part, v); }
};
template <bool BF16>
struct TgJob {
    const typename std::conditional<BF16, uint16_t, float>::type *dA, *P;
    BotArgs a;
    float* tbuf;
    static __device__ void run(const TgJob& j, int v) { bwd_t_gemm_body<BF16>(j.dA, j.P, j.a, j.tbuf, v); }
};
struct Dd1ReduceJob {
    const float* part;
    BotArgs a;
    int nsplit;
    float* dd1;
    static __device__ void run(const Dd1ReduceJob& j, int v) { bwd_dd1_reduce_body<float>(j.part, j.a, j.nsplit, j.dd1, v); }
};
struct Col2imJob {
    const float* tbuf;
    BotArgs a;
    float* dd2;
    static __device__ void run(const Col2imJob& j, int v) { bwd_col2im_body<float>(j.tbuf, j.a, j.dd2, v); }
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
    return a;
}

}  // namespace

int bwd_nsplit(const Geom& g) {
    // enough blocks for the 256 CUs: patch tiles x row splits >= ~1024
    const int ptiles = (g.gx[0] * g.gy[0] + G1P - 1) / G1P;
    int ns = (1024 + ptiles - 1) / ptiles;
    if (ns > g.H2) ns = g.H2;
    if (ns < 1) ns = 1;
    if (ns > 64) ns = 64;
    return ns;
}

size_t bwd_dense_bytes(const Geom& g, int precision) {
    const size_t es = precision == DM_BF16 ? 2 : 4;
    return (size_t)g.gx[0] * g.gy[0] * ((size_t)g.H2 * g.W2 + 144) * es;
}

// The six stages of the bottom backward of one pair as job records (FP32
// storage; bf16 selects BF16 MFMA operands), in launch order.
std::vector<JobRec> bot_jobs(bool bf16, const float* gp, const uint8_t* code, const float* d1, const float* d2,
                             const Geom& g, float* part, float* tbuf, void* dense, float* dd1, float* dd2) {
    const BotArgs a = make_bot(g);
    const int ns = bwd_nsplit(g);
    const int npos = a.H2 * a.W2;
    const int xblocks = (npos + 1023) / 1024;
    const int ptiles = (a.natom + G1P - 1) / G1P;
    const int tblocks = (npos + 127) / 128;
    const size_t pmat = (size_t)a.natom * 144;
    const int pm_blocks = (int)((pmat + 255) / 256);
    std::vector<JobRec> r(6);
    if (bf16) {
        uint16_t* dA = (uint16_t*)dense;
        uint16_t* P = dA + (size_t)a.natom * npos;
        r[0].set(JK_BWD_DA_BF16, a.natom * xblocks, 0, DaJob<uint16_t>{gp, code, a, xblocks, dA});
        r[1].set(JK_PATCH_BF16, pm_blocks, 0, PatchJob<uint16_t>{d1, a, P});
        r[2].set(JK_DD1_BF16, ptiles * ns, 0, Dd1Job<true>{dA, d2, a, ns, part});
        r[3].set(JK_TG_BF16, tblocks, 0, TgJob<true>{dA, P, a, tbuf});
    } else {
        float* dA = (float*)dense;
        float* P = dA + (size_t)a.natom * npos;
        r[0].set(JK_BWD_DA_F32, a.natom * xblocks, 0, DaJob<float>{gp, code, a, xblocks, dA});
        r[1].set(JK_PATCH_F32, pm_blocks, 0, PatchJob<float>{d1, a, P});
        r[2].set(JK_DD1_F32, ptiles * ns, 0, Dd1Job<false>{dA, d2, a, ns, part});
        r[3].set(JK_TG_F32, tblocks, 0, TgJob<false>{dA, P, a, tbuf});
    }
    const size_t n1 = (size_t)a.H1 * a.W1 * 9, n2 = (size_t)a.H2 * a.W2 * 9;
    r[4].set(JK_DD1_REDUCE, (int)((n1 + 255) / 256), 0, Dd1ReduceJob{part, a, ns, dd1});
    r[5].set(JK_COL2IM, (int)((n2 + 255) / 256), 0, Col2imJob{tbuf, a, dd2});
    return r;
}

hipError_t launch_group_bot(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_BWD_DA_BF16: return launch_grouped<DaJob<uint16_t>, 256, 1>(gl, s);
        case JK_BWD_DA_F32: return launch_grouped<DaJob<float>, 256, 1>(gl, s);
        case JK_PATCH_BF16: return launch_grouped<PatchJob<uint16_t>, 256, 1>(gl, s);
        case JK_PATCH_F32: return launch_grouped<PatchJob<float>, 256, 1>(gl, s);
        case JK_DD1_BF16: return launch_grouped<Dd1Job<true>, 256, 1>(gl, s);
        case JK_DD1_F32: return launch_grouped<Dd1Job<false>, 256, 1>(gl, s);
        case JK_TG_BF16: return launch_grouped<TgJob<true>, 256, 1>(gl, s);
        case JK_TG_F32: return launch_grouped<TgJob<false>, 256, 1>(gl, s);
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
    const BotArgs a = make_bot(g);
    int ns = 1;
    if (mode == 2) {  // reference kernels
        const size_t n1 = (size_t)a.natom * 144, n2 = (size_t)a.H2 * a.W2 * 144;
        DM_SUB("bwd_dd1_ref", k_bwd_dd1_ref<T>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, gp, code, d2, a, part);
        DM_SUB("bwd_t_ref", k_bwd_t_ref<T>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, gp, code, d1, a, tbuf);
    } else {
        if constexpr (std::is_same<T, float>::value) {
            ns = bwd_nsplit(g);
            const int npos = a.H2 * a.W2;
            const int xblocks = (npos + 1023) / 1024;
            const int ptiles = (a.natom + G1P - 1) / G1P;
            const int tblocks = (npos + 127) / 128;
            const size_t pmat = (size_t)a.natom * 144;
            if (mode == 1) {
                uint16_t* dA = (uint16_t*)dense;
                uint16_t* P = dA + (size_t)a.natom * npos;
                DM_SUB("bwd_da", k_bwd_da<uint16_t>, dim3(a.natom * xblocks), dim3(256), 0, s, gp, code, a, xblocks, dA);
                DM_SUB("bwd_patchmat", k_bwd_patchmat<uint16_t>, dim3((unsigned)((pmat + 255) / 256)), dim3(256), 0, s, d1, a, P);
                DM_SUB("bwd_dd1_gemm", k_bwd_dd1_gemm<true>, dim3(ptiles * ns), dim3(256), 0, s, dA, d2, a, ns, part);
                DM_SUB("bwd_t_gemm", k_bwd_t_gemm<true>, dim3(tblocks), dim3(256), 0, s, dA, P, a, tbuf);
            } else {
                float* dA = (float*)dense;
                float* P = dA + (size_t)a.natom * npos;
                DM_SUB("bwd_da", k_bwd_da<float>, dim3(a.natom * xblocks), dim3(256), 0, s, gp, code, a, xblocks, dA);
                DM_SUB("bwd_patchmat", k_bwd_patchmat<float>, dim3((unsigned)((pmat + 255) / 256)), dim3(256), 0, s, d1, a, P);
                DM_SUB("bwd_dd1_gemm", k_bwd_dd1_gemm<false>, dim3(ptiles * ns), dim3(256), 0, s, dA, d2, a, ns, part);
                DM_SUB("bwd_t_gemm", k_bwd_t_gemm<false>, dim3(tblocks), dim3(256), 0, s, dA, P, a, tbuf);
            }
        } else {
            return hipErrorInvalidValue;
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n1 = (size_t)a.H1 * a.W1 * 9, n2 = (size_t)a.H2 * a.W2 * 9;
    DM_SUB("bwd_dd1_reduce", k_bwd_dd1_reduce<T>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, part, a, ns, dd1);
    DM_SUB("bwd_col2im", k_bwd_col2im<T>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, tbuf, a, dd2);
    return hipGetLastError();
#undef DM_SUB
}

template hipError_t launch_bwd_bottom<float>(int, const float*, const uint8_t*, const float*, const float*,
                                             const Geom&, float*, float*, void*, float*, float*, hipStream_t);
template hipError_t launch_bwd_bottom<double>(int, const double*, const uint8_t*, const double*, const double*,
                                              const Geom&, double*, double*, void*, double*, double*, hipStream_t);

}  // namespace dm
