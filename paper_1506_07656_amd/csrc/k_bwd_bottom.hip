// Adjoint of the bottom correlation (Eq. (3)) for the gradient pass.
//
// With g'_0(p, r) the gradient routed to pooled entry r of atomic patch p
// (see k_backward.hip), the gradient with respect to A_0 is
//   dA_0(p, x) = sum_{r: 2r + m_0(p, r) = x} g'_0(p, r)        (<= 4 candidates)
// and, with K index k = (dy, dx, c) over the 4x4 patch and 9 channels,
//   dD1[p + d_k][c_k] = 1/16 sum_x dA_0(p, x) D2[x + d_k][c_k]          (GEMM 1)
//   T[x][k]           =      sum_p dA_0(p, x) D1[p + d_k][c_k]          (GEMM 2)
//   dD2[y][c]         = 1/16 sum_{dy,dx} T[y - d][(d, c)]               (col2im)
// Atomic patches do not overlap, so GEMM 1 writes each D1 pixel once.  Both
// GEMMs run on the matrix cores with dA_0 rebuilt tile by tile in LDS from
// g'_0 and the argmax codes (never stored densely); partial sums over split
// ranges are added in a fixed order, so the result is deterministic.
//
// Reference kernels (thread per output, direct loops) serve the FP64
// instantiation used by the finite-difference check.
#include <type_traits>

#include "dm_internal.h"

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

// ---------------------------------------------------------------- GEMM 1: dD1
// Block: 64 patches (16 per wave) x all 144 K columns (9 N-tiles); it reduces
// over the positions of one split.  Each chunk of 64 positions rebuilds the
// dA tile [64 patches][64 positions] and the im2col tile [144][64 positions]
// in LDS (operand type E: float or bf16), then runs the MFMA chain.
constexpr int BP = 64, KC = 64;

template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_dd1_mfma(const float* __restrict__ gp, const uint8_t* __restrict__ code,
                                                      const float* __restrict__ d2, BotArgs a, int nsplit,
                                                      float* __restrict__ part) {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    __shared__ __align__(16) E sA[BP][KC + (BF16 ? 8 : 1)];
    __shared__ __align__(16) E sB[144][KC + (BF16 ? 8 : 1)];
    const int ptile = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    const int npos = a.H2 * a.W2;
    const int per = (npos + nsplit - 1) / nsplit;
    const int x_begin = split * per, x_end = min(npos, x_begin + per);
    const size_t pm = (size_t)a.h1 * a.w1;
    f4 acc[9];
#pragma unroll
    for (int nt = 0; nt < 9; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int x0 = x_begin; x0 < x_end; x0 += KC) {
        __syncthreads();
        for (int e = tid; e < BP * KC; e += 256) {
            const int pl = e / KC, xi = e - pl * KC;
            const int p = ptile * BP + pl, xl = x0 + xi;
            float v = 0.f;
            if (p < a.natom && xl < x_end) {
                const int xy = xl / a.W2, xx = xl - xy * a.W2;
                v = dA_at(gp + p * pm, code + p * pm, a.h1, a.w1, xy, xx);
            }
            if constexpr (BF16) sA[pl][xi] = to_bf16(v); else sA[pl][xi] = v;
        }
        for (int e = tid; e < 144 * KC; e += 256) {
            const int k = e / KC, xi = e - k * KC;
            const int xl = x0 + xi;
            float v = 0.f;
            if (xl < x_end) {
                const int xy = xl / a.W2, xx = xl - xy * a.W2;
                v = d2_at(d2, a, xy, xx, k);
            }
            if constexpr (BF16) sB[k][xi] = to_bf16(v); else sB[k][xi] = v;
        }
        __syncthreads();
        const int pr = wave * 16 + n;
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < KC / 32; ++s) {
                const bf8 av = as_bf8(&sA[pr][32 * s + 8 * g]);
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const bf8 bv = as_bf8(&sB[16 * nt + n][32 * s + 8 * g]);
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 4
            for (int t = 0; t < KC / 4; ++t) {
                const float av = sA[pr][4 * t + g];
#pragma unroll
                for (int nt = 0; nt < 9; ++nt)
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sB[16 * nt + n][4 * t + g], acc[nt], 0, 0, 0);
            }
        }
    }
    // acc[nt][j]: patch wave*16 + 4g + j, column 16 nt + n
#pragma unroll
    for (int nt = 0; nt < 9; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = ptile * BP + wave * 16 + 4 * g + j;
            if (p < a.natom) part[((size_t)split * a.natom + p) * 144 + 16 * nt + n] = acc[nt][j];
        }
}

// dD1 (HWC) from the split partials: each pixel belongs to at most one patch.
template <typename T>
__global__ void k_bwd_dd1_reduce(const T* __restrict__ part, BotArgs a, int nsplit, T* __restrict__ dd1) {
    const size_t n = (size_t)a.H1 * a.W1 * 9;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
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
// Block: 64 positions (16 per wave) x 144 columns; reduces over all patches
// in chunks of 64: dA tile [64 patches][64 positions] and patch tile
// [144][64 patches] in LDS.
template <bool BF16>
__global__ __launch_bounds__(256) void k_bwd_t_mfma(const float* __restrict__ gp, const uint8_t* __restrict__ code,
                                                    const float* __restrict__ d1, BotArgs a, float* __restrict__ tbuf) {
    typedef typename std::conditional<BF16, uint16_t, float>::type E;
    __shared__ __align__(16) E sA[64][64 + (BF16 ? 8 : 1)];     // [position][patch]
    __shared__ __align__(16) E sB[144][64 + (BF16 ? 8 : 1)];    // [k][patch]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, n = lane & 15, g = lane >> 4;
    const int npos = a.H2 * a.W2;
    const int xb = blockIdx.x * 64;
    const size_t pm = (size_t)a.h1 * a.w1;
    f4 acc[9];
#pragma unroll
    for (int nt = 0; nt < 9; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < a.natom; p0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += 256) {
            const int xi = e / 64, pl = e - xi * 64;
            const int p = p0 + pl, xl = xb + xi;
            float v = 0.f;
            if (p < a.natom && xl < npos) {
                const int xy = xl / a.W2, xx = xl - xy * a.W2;
                v = dA_at(gp + p * pm, code + p * pm, a.h1, a.w1, xy, xx);
            }
            if constexpr (BF16) sA[xi][pl] = to_bf16(v); else sA[xi][pl] = v;
        }
        for (int e = tid; e < 144 * 64; e += 256) {
            const int pl = e / 144, k = e - pl * 144;
            const int p = p0 + pl;
            const float v = p < a.natom ? d1_at(d1, a, p, k) : 0.f;
            if constexpr (BF16) sB[k][pl] = to_bf16(v); else sB[k][pl] = v;
        }
        __syncthreads();
        const int xr = wave * 16 + n;
        if constexpr (BF16) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bf8 av = as_bf8(&sA[xr][32 * s + 8 * g]);
#pragma unroll
                for (int nt = 0; nt < 9; ++nt) {
                    const bf8 bv = as_bf8(&sB[16 * nt + n][32 * s + 8 * g]);
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll 4
            for (int t = 0; t < 16; ++t) {
                const float av = sA[xr][4 * t + g];
#pragma unroll
                for (int nt = 0; nt < 9; ++nt)
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sB[16 * nt + n][4 * t + g], acc[nt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int nt = 0; nt < 9; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xl = xb + wave * 16 + 4 * g + j;
            if (xl < npos) tbuf[(size_t)xl * 144 + 16 * nt + n] = acc[nt][j];
        }
}

// dD2[y][c] = 1/16 sum_d T[y - d][(d, c)]  (T is zero outside the target).
template <typename T>
__global__ void k_bwd_col2im(const T* __restrict__ tbuf, BotArgs a, T* __restrict__ dd2) {
    const size_t n = (size_t)a.H2 * a.W2 * 9;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    // enough blocks for the 256 CUs: patch tiles x splits >= ~1024
    const int ptiles = (g.gx[0] * g.gy[0] + BP - 1) / BP;
    int ns = (1024 + ptiles - 1) / ptiles;
    const int npos = g.H2 * g.W2;
    const int maxs = (npos + KC - 1) / KC;
    if (ns > maxs) ns = maxs;
    if (ns < 1) ns = 1;
    if (ns > 64) ns = 64;
    return ns;
}

template <typename T>
hipError_t launch_bwd_bottom(int mode, const T* gp, const uint8_t* code, const T* d1, const T* d2, const Geom& g,
                             T* part, T* tbuf, T* dd1, T* dd2, hipStream_t s) {
    const BotArgs a = make_bot(g);
    int ns = 1;
    if (mode == 2) {  // reference kernels
        const size_t n1 = (size_t)a.natom * 144, n2 = (size_t)a.H2 * a.W2 * 144;
        hipLaunchKernelGGL(k_bwd_dd1_ref<T>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, gp, code, d2, a, part);
        hipLaunchKernelGGL(k_bwd_t_ref<T>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, gp, code, d1, a, tbuf);
    } else {
        if constexpr (std::is_same<T, float>::value) {
            ns = bwd_nsplit(g);
            const int ptiles = (a.natom + BP - 1) / BP;
            const int tblocks = (a.H2 * a.W2 + 63) / 64;
            if (mode == 1) {
                hipLaunchKernelGGL(k_bwd_dd1_mfma<true>, dim3(ptiles * ns), dim3(256), 0, s, gp, code, d2, a, ns, part);
                hipLaunchKernelGGL(k_bwd_t_mfma<true>, dim3(tblocks), dim3(256), 0, s, gp, code, d1, a, tbuf);
            } else {
                hipLaunchKernelGGL(k_bwd_dd1_mfma<false>, dim3(ptiles * ns), dim3(256), 0, s, gp, code, d2, a, ns, part);
                hipLaunchKernelGGL(k_bwd_t_mfma<false>, dim3(tblocks), dim3(256), 0, s, gp, code, d1, a, tbuf);
            }
        } else {
            return hipErrorInvalidValue;
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n1 = (size_t)a.H1 * a.W1 * 9, n2 = (size_t)a.H2 * a.W2 * 9;
    hipLaunchKernelGGL(k_bwd_dd1_reduce<T>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, part, a, ns, dd1);
    hipLaunchKernelGGL(k_bwd_col2im<T>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, tbuf, a, dd2);
    return hipGetLastError();
}

template hipError_t launch_bwd_bottom<float>(int, const float*, const uint8_t*, const float*, const float*,
                                             const Geom&, float*, float*, float*, float*, hipStream_t);
template hipError_t launch_bwd_bottom<double>(int, const double*, const uint8_t*, const double*, const double*,
                                              const Geom&, double*, double*, double*, double*, hipStream_t);

}  // namespace dm
