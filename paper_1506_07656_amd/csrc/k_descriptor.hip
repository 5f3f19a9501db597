// Per-pixel descriptor (Sec. 3.2, "Pixel descriptor"), one fused kernel.
//
// Each block produces a TX x TY tile of descriptors.  The chain of stencils
// (optional smoothing nu1, central-difference gradient, 8 non-negative
// orientation projections, smoothing nu2, sigmoid cap, smoothing nu3,
// l2-normalisation with the constant mu) runs in LDS on regions that shrink
// by each stage's radius.  Borders replicate: every LDS entry holds the value
// of its stage at the CLAMPED image position, and reads clamp again, so a
// stage never needs values outside the image.
#include "dm_group.h"

namespace dm {
namespace {

constexpr int TX = 32, TY = 16, NT = 256;

struct Region {
    int ox, oy, w, h;  // image-space origin and size
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// cos and sin of k*pi/4 for k = 1..8 (y down).
__constant__ float kCos[8] = {0.70710678118654752f, 0.f, -0.70710678118654752f, -1.f,
                              -0.70710678118654752f, 0.f, 0.70710678118654752f, 1.f};
__constant__ float kSin[8] = {0.70710678118654752f, 1.f, 0.70710678118654752f, 0.f,
                              -0.70710678118654752f, -1.f, -0.70710678118654752f, 0.f};

__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

__device__ inline void descriptor_body(const float* __restrict__ img, int W, int H, int ld, const DescParams& p,
                                       float* __restrict__ out, uint16_t* __restrict__ out_bf, int bx, int by) {
    extern __shared__ float smem[];
    const int x0 = bx * TX, y0 = by * TY;
    const int r1 = p.r1, r2 = p.r2, r3 = p.r3;
    const int tid = threadIdx.x;
    // Regions, from the output tile outwards.
    const Region Rx3 = {x0, y0 - r3, TX, TY + 2 * r3};                               // nu3 x-pass out
    const Region Rs = {x0 - r3, y0 - r3, TX + 2 * r3, TY + 2 * r3};                   // sigmoid (nu2 y-pass out)
    const Region Rx2 = {Rs.ox, Rs.oy - r2, Rs.w, Rs.h + 2 * r2};                       // nu2 x-pass out
    const Region Ro = {Rs.ox - r2, Rs.oy - r2, Rs.w + 2 * r2, Rs.h + 2 * r2};          // orientation maps
    const Region Rj = {Ro.ox - 1, Ro.oy - 1, Ro.w + 2, Ro.h + 2};                      // intensities (smoothed)
    const Region Rjx = {Rj.ox, Rj.oy - r1, Rj.w, Rj.h + 2 * r1};                       // nu1 x-pass out
    const Region Rraw = {Rj.ox - r1, Rj.oy - r1, Rj.w + 2 * r1, Rj.h + 2 * r1};        // raw intensities
    // LDS: buf0 holds the 8-channel orientation maps, later the sigmoid maps;
    // buf1 holds the intensity stages, later the nu2 and nu3 x-pass outputs.
    float* buf0 = smem;
    float* buf1 = smem + 8 * Ro.w * Ro.h;
    const int n_raw = Rraw.w * Rraw.h, n_jx = Rjx.w * Rjx.h;
    float* sraw = buf1;
    float* sjx = buf1 + n_raw;
    float* sj = r1 ? buf1 + n_raw + n_jx : buf1;

    auto at = [&](const Region& R, int X, int Y) {  // LDS index of clamped image position
        return (clampi(Y, 0, H - 1) - R.oy) * R.w + (clampi(X, 0, W - 1) - R.ox);
    };

    // Stage 1: intensities (scaled), optionally smoothed with nu1.
    float* jdst = r1 ? sraw : sj;
    const Region& Rjdst = r1 ? Rraw : Rj;
    for (int e = tid; e < Rjdst.w * Rjdst.h; e += NT) {
        const int X = clampi(Rjdst.ox + e % Rjdst.w, 0, W - 1), Y = clampi(Rjdst.oy + e / Rjdst.w, 0, H - 1);
        jdst[e] = p.scale * img[(size_t)Y * ld + X];
    }
    __syncthreads();
    if (r1) {
        for (int e = tid; e < n_jx; e += NT) {
            const int X = clampi(Rjx.ox + e % Rjx.w, 0, W - 1), Y = clampi(Rjx.oy + e / Rjx.w, 0, H - 1);
            float acc = 0.f;
            for (int t = -r1; t <= r1; ++t) acc += p.g1[t + r1] * sraw[at(Rraw, X + t, Y)];
            sjx[e] = acc;
        }
        __syncthreads();
        for (int e = tid; e < Rj.w * Rj.h; e += NT) {
            const int X = clampi(Rj.ox + e % Rj.w, 0, W - 1), Y = clampi(Rj.oy + e / Rj.w, 0, H - 1);
            float acc = 0.f;
            for (int t = -r1; t <= r1; ++t) acc += p.g1[t + r1] * sjx[at(Rjx, X, Y + t)];
            sj[e] = acc;
        }
        __syncthreads();
    }
    // Stage 2: gradient by central differences, 8 non-negative projections.
    const int n_o = Ro.w * Ro.h;
    for (int e = tid; e < n_o; e += NT) {
        const int X = clampi(Ro.ox + e % Ro.w, 0, W - 1), Y = clampi(Ro.oy + e / Ro.w, 0, H - 1);
        const float gx = 0.5f * (sj[at(Rj, X + 1, Y)] - sj[at(Rj, X - 1, Y)]);
        const float gy = 0.5f * (sj[at(Rj, X, Y + 1)] - sj[at(Rj, X, Y - 1)]);
#pragma unroll
        for (int k = 0; k < 8; ++k) buf0[k * n_o + e] = fmaxf(0.f, gx * kCos[k] + gy * kSin[k]);
    }
    __syncthreads();
    // Stage 3: smoothing nu2 (x then y), sigmoid cap.
    const int n_x2 = Rx2.w * Rx2.h;
    for (int e = tid; e < n_x2; e += NT) {
        const int X = clampi(Rx2.ox + e % Rx2.w, 0, W - 1), Y = clampi(Rx2.oy + e / Rx2.w, 0, H - 1);
        for (int k = 0; k < 8; ++k) {
            float acc = 0.f;
            for (int t = -r2; t <= r2; ++t) acc += p.g2[t + r2] * buf0[k * n_o + at(Ro, X + t, Y)];
            buf1[k * n_x2 + e] = acc;
        }
    }
    __syncthreads();
    const int n_s = Rs.w * Rs.h;
    for (int e = tid; e < n_s; e += NT) {
        const int X = clampi(Rs.ox + e % Rs.w, 0, W - 1), Y = clampi(Rs.oy + e / Rs.w, 0, H - 1);
        for (int k = 0; k < 8; ++k) {
            float acc = 0.f;
            for (int t = -r2; t <= r2; ++t) acc += p.g2[t + r2] * buf1[k * n_x2 + at(Rx2, X, Y + t)];
            buf0[k * n_s + e] = 2.f / (1.f + __expf(-p.slope * acc)) - 1.f;
        }
    }
    __syncthreads();
    // Stage 4: smoothing nu3, x-pass.
    const int n_x3 = Rx3.w * Rx3.h;
    for (int e = tid; e < n_x3; e += NT) {
        const int X = clampi(Rx3.ox + e % Rx3.w, 0, W - 1), Y = clampi(Rx3.oy + e / Rx3.w, 0, H - 1);
        for (int k = 0; k < 8; ++k) {
            float acc = 0.f;
            for (int t = -r3; t <= r3; ++t) acc += p.g3[t + r3] * buf0[k * n_s + at(Rs, X + t, Y)];
            buf1[k * n_x3 + e] = acc;
        }
    }
    __syncthreads();
    // Stage 5: nu3 y-pass, append mu, l2-normalise, store.
    for (int e = tid; e < TX * TY; e += NT) {
        const int X = x0 + e % TX, Y = y0 + e / TX;
        if (X >= W || Y >= H) continue;
        float v[9];
        float ss = p.mu * p.mu;
        for (int k = 0; k < 8; ++k) {
            float acc = 0.f;
            for (int t = -r3; t <= r3; ++t) acc += p.g3[t + r3] * buf1[k * n_x3 + at(Rx3, X, Y + t)];
            v[k] = acc;
            ss += acc * acc;
        }
        v[8] = p.mu;
        const float inv = 1.f / sqrtf(ss);
        float* o = out + ((size_t)Y * W + X) * 9;
        for (int k = 0; k < 9; ++k) o[k] = v[k] * inv;
        if (out_bf) {
            uint16_t* ob = out_bf + ((size_t)Y * W + X) * 10;
            for (int k = 0; k < 9; ++k) ob[k] = to_bf16(v[k] * inv);
            ob[9] = 0;
        }
    }
}

__global__ __launch_bounds__(NT) void k_descriptor(const float* __restrict__ img, int W, int H, int ld,
                                                   DescParams p, float* __restrict__ out,
                                                   uint16_t* __restrict__ out_bf) {
    descriptor_body(img, W, H, ld, p, out, out_bf, blockIdx.x, blockIdx.y);
}

struct DescJob {
    const float* img;
    int W, H, ld, gx;
    float* out;
    uint16_t* out_bf;
    DescParams p;
    static __device__ void run(const DescJob& j, int v) {
        const int by = v / j.gx;
        descriptor_body(j.img, j.W, j.H, j.ld, j.p, j.out, j.out_bf, v - by * j.gx, by);
    }
};

// FP32 HWC (9 channels) -> BF16 with a zero 10th channel.
__global__ void k_to_bf16(const float* __restrict__ d, int n_pix, uint16_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pix * 10) return;
    const int px = i / 10, c = i % 10;
    out[i] = c < 9 ? to_bf16(d[(size_t)px * 9 + c]) : (uint16_t)0;
}

}  // namespace

static size_t desc_smem_bytes(const DescParams& p) {
    const int r1 = p.r1, r2 = p.r2, r3 = p.r3;
    const int sw = TX + 2 * r3, sh = TY + 2 * r3;
    const int ow = sw + 2 * r2, oh = sh + 2 * r2;
    const int jw = ow + 2, jh = oh + 2;
    const size_t b0 = (size_t)8 * ow * oh;
    size_t b1 = (size_t)8 * sw * (sh + 2 * r2);
    const size_t x3 = (size_t)8 * TX * sh;
    if (x3 > b1) b1 = x3;
    const size_t js = r1 ? (size_t)(jw + 2 * r1) * (jh + 2 * r1) + (size_t)jw * (jh + 2 * r1) + (size_t)jw * jh
                         : (size_t)jw * jh;
    if (js > b1) b1 = js;
    return (b0 + b1) * sizeof(float);
}

hipError_t launch_descriptor(const float* img, int W, int H, int ld, const DescParams& p, float* out,
                             uint16_t* out_bf16, hipStream_t s) {
    const dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY);
    const size_t smem = desc_smem_bytes(p);
    if (smem > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_descriptor, grid, dim3(NT), smem, s, img, W, H, ld, p, out, out_bf16);
    return hipGetLastError();
}

// Both images of a pair in one launch (blockIdx.z picks the image): each
// image alone fills only one block per CU, as a block's stencil stages need
// most of the LDS.  The per-image fields are selected one by one (selecting
// between two by-value structs would put them in scratch memory).
struct DescImage {
    const float* img;
    int W, H, ld;
    float* out;
    uint16_t* out_bf;
};

__global__ __launch_bounds__(NT) void k_descriptor_pair(DescImage i0, DescImage i1, DescParams p) {
    const bool second = blockIdx.z != 0;
    const int W = second ? i1.W : i0.W, H = second ? i1.H : i0.H;
    if ((int)blockIdx.x * TX >= W || (int)blockIdx.y * TY >= H) return;
    descriptor_body(second ? i1.img : i0.img, W, H, second ? i1.ld : i0.ld, p, second ? i1.out : i0.out,
                    second ? i1.out_bf : i0.out_bf, blockIdx.x, blockIdx.y);
}

hipError_t launch_descriptor_pair(const float* img1, int W1, int H1, int ld1, float* out1, uint16_t* bf1,
                                  const float* img2, int W2, int H2, int ld2, float* out2, uint16_t* bf2,
                                  const DescParams& p, hipStream_t s) {
    const DescImage i0{img1, W1, H1, ld1, out1, bf1}, i1{img2, W2, H2, ld2, out2, bf2};
    const dim3 grid(((W1 > W2 ? W1 : W2) + TX - 1) / TX, ((H1 > H2 ? H1 : H2) + TY - 1) / TY, 2);
    const size_t smem = desc_smem_bytes(p);
    if (smem > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_descriptor_pair, grid, dim3(NT), smem, s, i0, i1, p);
    return hipGetLastError();
}

JobRec desc_job(const float* img, int W, int H, int ld, const DescParams& p, float* out, uint16_t* out_bf16) {
    DescJob j{img, W, H, ld, (W + TX - 1) / TX, out, out_bf16, p};
    JobRec r;
    r.set(JK_DESC, j.gx * ((H + TY - 1) / TY), desc_smem_bytes(p), j);
    return r;
}

hipError_t launch_group_desc(int kind, const GroupLaunch& gl, hipStream_t s) {
    if (kind != JK_DESC) return hipErrorInvalidValue;
    return launch_grouped<DescJob, NT, 1>(gl, s);
}

hipError_t launch_to_bf16(const float* d, int n_pix, uint16_t* out, hipStream_t s) {
    const int n = n_pix * 10;
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, s, d, n_pix, out);
    return hipGetLastError();
}

}  // namespace dm
