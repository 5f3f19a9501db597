// Approximate DeepMatching (Sec. 4.1): spherical k-means over the atomic
// patches of I, and the prototypes laid out as a small image (4 rows, 4D
// columns) whose D atomic patches are the prototypes, so that the bottom
// correlation kernels compute the D prototype maps C'_0 unchanged.
//
// A patch vector is the 16 pixel descriptors of its 4x4 patch in (dy, dx,
// channel) order (144 values, norm 4).  Centroid d starts as patch
// floor((2d+1) n / (2D)); each iteration assigns every patch to the centroid
// with the largest dot product (values within kTie of the largest count as
// equal, lowest index first), then replaces every centroid that has members
// by the sum of its members rescaled to norm 4; a final assignment follows.
//
// Every decision is the one an FP64 evaluation takes:
//  * Assignment.  FP32 MFMA dot products of all patches with all centroids;
//    each patch keeps its two best (value, index) pairs and the best value
//    after them.  Descriptors and centroids are non-negative and of norm 4,
//    so a 144-term FP32 dot product (at most 16) is within
//    gamma_145 * 16 + 16 u < 1.4e-4 of the exact one (u = 2^-24), whatever
//    the summation order.  With kGap = 5e-4 > 2 * 1.4e-4 + kTie:
//      v1 - v2 > kGap:  the best centroid is the FP64 answer;
//      v1 - v3 > kGap:  the answer is one of the two best, decided in FP64;
//      otherwise:       every centroid is evaluated in FP64.
//  * Update.  Member sums in FP64, in a fixed order, then the norm and the
//    rescale in FP64.  Results are deterministic run to run.
#include <math.h>

#include "dm_group.h"

namespace dm {
namespace {

constexpr double kTie = 1e-11;     // dot products this close to the largest are equal
constexpr float kGap = 5e-4f;      // FP32 gap that certifies a decision (see above)
constexpr int KM_LD = 148;         // LDS row stride (floats) of a staged centroid
constexpr int KM_FIX = 64;         // patches per block of the decision kernel (one wave)
constexpr int KM_G3 = 16;          // patches per group of the all-centroid FP64 path

typedef float f4 __attribute__((ext_vector_type(4)));

// Element k of the vector of atomic patch p (lattice gx0 wide).
__device__ inline float patch_elem(const KmArgs& a, int p, int k) {
    const int b = p / a.gx0, aa = p - b * a.gx0;
    const int r = k / 36, j = k - r * 36;
    return a.d1[((size_t)(4 * b + r) * a.W1 + 4 * aa) * 9 + j];
}

__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

// Sum over the 64 lanes by a butterfly: every lane ends with the same value
// (each pairwise sum is computed identically on both lanes of the pair).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Order-independent hash of a centroid: the XOR over its elements of a
// mixed (value bits, element index), reduced over the wave.
__device__ inline unsigned long long elem_hash(double v, int k) {
    unsigned long long z = (unsigned long long)__double_as_longlong(v) ^ (0x9E3779B97F4A7C15ull * (k + 1));
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline unsigned long long wave_xor(unsigned long long h) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)h, m), hi = __shfl_xor((uint32_t)(h >> 32), m);
        h ^= ((unsigned long long)hi << 32) | lo;
    }
    return h;
}

// Writes element k of centroid d: the FP64 value, and its FP32 and BF16 forms
// at pixel (row k / 36, column 4d + (k % 36) / 9) of the prototype image.
__device__ inline void put_centroid(const KmArgs& a, int d, int k, double v) {
    a.C64[(size_t)d * 144 + k] = v;
    a.C64T[(size_t)k * a.D + d] = v;
    const int r = k / 36, j = k - r * 36;
    a.img[(size_t)r * 36 * a.D + 36 * d + j] = (float)v;
    if (a.img16) {
        const int dx = j / 9, c = j - dx * 9;
        a.img16[((size_t)r * 4 * a.D + 4 * d + dx) * 10 + c] = bf16_rne((float)v);
    }
}

// One wave per centroid: the starting patch rescaled to norm 4.
__global__ __launch_bounds__(64) void k_km_init(KmArgs a) {
    const int d = blockIdx.x, lane = threadIdx.x;
    if (d == 0 && lane < 2) a.stat[lane] = 0;
    const int p = (int)(((2ll * d + 1) * a.n) / (2ll * a.D));
    double v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = lane + 64 * i;
        v[i] = k < 144 ? (double)patch_elem(a, p, k) : 0.0;
    }
    const double n2 = wave_sum(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double sc = n2 > 0.0 ? 4.0 / sqrt(n2) : 0.0;
    unsigned long long h = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = lane + 64 * i;
        if (k < 144) {
            put_centroid(a, d, k, v[i] * sc);
            h ^= elem_hash(v[i] * sc, k);
        }
    }
    h = wave_xor(h);
    if (lane == 0) a.hash[d] = h;
    if (a.img16 && lane < 16) {   // the padding channel of the prototype's 16 pixels
        const int r = lane >> 2, dx = lane & 3;
        a.img16[((size_t)r * 4 * a.D + 4 * d + dx) * 10 + 9] = 0;
    }
}

// Shadowed centroids: d is shadowed when it equals (all 144 FP64 values) a
// centroid of lower index.  Its dot products then equal that centroid's in
// any evaluation, so the tie rule never chooses it: both assignment paths
// skip it.  Hashes are compared first; equal hashes are confirmed element by
// element.
__global__ __launch_bounds__(256) void k_km_shadow(KmArgs a) {
    const int d = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (d >= a.D) return;
    const unsigned long long h = a.hash[d];
    bool sh = false;   // uniform over the wave
    for (int e0 = 0; e0 < d && !sh; e0 += 64) {
        const int e = e0 + lane;
        unsigned long long m = __ballot(e < d && a.hash[e] == h);
        while (m && !sh) {
            const int ee = e0 + __ffsll((long long)m) - 1;
            m &= m - 1;
            bool diff = false;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int k = lane + 64 * i;
                if (k < 144) diff |= a.C64[(size_t)ee * 144 + k] != a.C64[(size_t)d * 144 + k];
            }
            sh = __ballot(diff) == 0ull;
        }
    }
    if (lane == 0) a.shadow[d] = sh ? 1 : 0;
}

// Best two (value, index) pairs and the best value after them.
struct Top3 {
    float v1, v2, v3;
    int i1, i2;
};

__device__ inline void push(Top3& s, float v, int d) {
    if (v > s.v1) {
        s.v3 = s.v2;
        s.v2 = s.v1;
        s.i2 = s.i1;
        s.v1 = v;
        s.i1 = d;
    } else if (v > s.v2) {
        s.v3 = s.v2;
        s.v2 = v;
        s.i2 = d;
    } else if (v > s.v3) {
        s.v3 = v;
    }
}

__device__ inline void merge(Top3& s, const Top3& o) {
    push(s, o.v1, o.i1);
    push(s, o.v2, o.i2);
    s.v3 = fmaxf(s.v3, o.v3);
}

// A chunk's Top3 as one 16-byte record: the three values and both indices
// (below 2^16; 0xFFFF = none) in the fourth word.
__device__ inline f4 pack(const Top3& s) {
    const uint32_t i = (uint32_t)min(s.i1, 0xFFFF) | ((uint32_t)min(s.i2, 0xFFFF) << 16);
    return f4{s.v1, s.v2, s.v3, __uint_as_float(i)};
}
__device__ inline Top3 unpack(const f4 r) {
    const uint32_t i = __float_as_uint(r[3]);
    return Top3{r[0], r[1], r[2], (int)(i & 0xFFFF), (int)(i >> 16)};
}

__device__ inline Top3 shfl_xor_top3(const Top3& s, int m) {
    Top3 o;
    o.v1 = __shfl_xor(s.v1, m);
    o.v2 = __shfl_xor(s.v2, m);
    o.v3 = __shfl_xor(s.v3, m);
    o.i1 = __shfl_xor(s.i1, m);
    o.i2 = __shfl_xor(s.i2, m);
    return o;
}

// FP32 pass: block (patch block, centroid chunk of KM_CH); NT = 2 patch
// tiles per wave where that still makes two blocks per compute unit (many
// centroids), else 1 (twice the blocks: with 64 centroids the 2-tile grid
// has 64 blocks, and its launch takes 1.3 times as long).  The chunk's
// centroids are staged in LDS; each wave keeps NT tiles of 16 patches in
// registers as the B operand of v_mfma_f32_16x16x4f32 (K = 144 split so that
// the 16-lane group g of a wave owns the 36 values of patch row g, one
// contiguous run in both layouts) and takes the centroids 16 at a time as the
// A operand.  Lane (g, n) receives centroids 4g..4g+3 of the tile for patch
// n and folds them into its running Top3.
template <int NT>
__global__ __launch_bounds__(256) void k_km_assign(KmArgs a) {
    constexpr int PB = 64 * NT;   // patches per block (4 waves)
    __shared__ __align__(16) float sC[KM_CH * KM_LD];
    __shared__ int sSh[KM_CH];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, grp = lane >> 4;
    const int chunk = blockIdx.y, d0 = chunk * KM_CH;
    const int nd = min(KM_CH, a.D - d0);
    // 16-byte pieces: centroid i, patch row r, piece v (9 per row of 36 floats)
    for (int e = tid; e < KM_CH * 36; e += 256) {
        const int i = e / 36, rv = e - i * 36, r = rv / 9, v = rv - r * 9;
        f4 x = f4{0.f, 0.f, 0.f, 0.f};
        if (i < nd) x = *(const f4*)(a.img + (size_t)r * 36 * a.D + 36 * (d0 + i) + 4 * v);
        *(f4*)(sC + i * KM_LD + 36 * r + 4 * v) = x;
    }
    if (tid < KM_CH) sSh[tid] = tid < nd ? a.shadow[d0 + tid] : 1;
    float fb[NT][36];
    int pp[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int p = blockIdx.x * PB + wave * 16 * NT + nt * 16 + n;
        pp[nt] = p;
        if (p < a.n) {
            const int b = p / a.gx0, aa = p - b * a.gx0;
            const float* src = a.d1 + ((size_t)(4 * b + grp) * a.W1 + 4 * aa) * 9;
#pragma unroll
            for (int t = 0; t < 36; ++t) fb[nt][t] = src[t];
        } else {
#pragma unroll
            for (int t = 0; t < 36; ++t) fb[nt][t] = 0.f;
        }
    }
    __syncthreads();
    Top3 st[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) st[nt] = Top3{-INFINITY, -INFINITY, -INFINITY, 0x7fffffff, 0x7fffffff};
    for (int ct = 0; ct * 16 < nd; ++ct) {
        const float* src = sC + (ct * 16 + n) * KM_LD + grp * 36;
        f4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 36; ++t) {
            const float fa = src[t];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, fb[nt][t], acc[nt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ct * 16 + 4 * grp + r;
                if (!sSh[i]) push(st[nt], acc[nt][r], d0 + i);   // i >= nd is marked shadowed
            }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        merge(st[nt], shfl_xor_top3(st[nt], 16));
        merge(st[nt], shfl_xor_top3(st[nt], 32));
        const int p = pp[nt];
        if (grp == 0 && p < a.n) a.part[(size_t)chunk * a.n + p] = pack(st[nt]);
    }
}

// Dot products of centroid d with the KM_G3 rows of sX, FP64 FMAs in k
// order; the centroid's column is read KM_KB values at a time so that the
// loads are in flight together.
constexpr int KM_KB = 24;
__device__ inline void dots_g3(const KmArgs& a, int d, const double (*sX)[144], double (&t)[KM_G3]) {
    for (int k0 = 0; k0 < 144; k0 += KM_KB) {
        double c[KM_KB];
#pragma unroll
        for (int u = 0; u < KM_KB; ++u) c[u] = a.C64T[(size_t)(k0 + u) * a.D + d];
#pragma unroll
        for (int u = 0; u < KM_KB; ++u)
#pragma unroll
            for (int j = 0; j < KM_G3; ++j) t[j] = fma(sX[j][k0 + u], c[u], t[j]);
    }
}

// Decisions: merge the chunks' Top3 of each patch (fixed order), keep
// certified answers, and settle the others in FP64 (two candidates: one wave
// per patch; more: the whole block per patch, over every centroid).
__global__ __launch_bounds__(KM_FIX) void k_km_fix(KmArgs a) {
    __shared__ int sP2[KM_FIX], sA2[KM_FIX], sB2[KM_FIX], sP3[KM_FIX];
    __shared__ int sN2, sN3;
    __shared__ double sX[KM_G3][144];
    __shared__ double sRed[KM_G3][KM_FIX / 64];
    __shared__ int sRedI[KM_G3][KM_FIX / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) sN2 = sN3 = 0;
    __syncthreads();
    const int p = blockIdx.x * KM_FIX + tid;
    if (p < a.n) {
        Top3 s = unpack(a.part[p]);
        for (int c0 = 1; c0 < a.nchunk; c0 += 4) {   // four chunks' loads in flight, merged in order
            f4 r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + u < a.nchunk) r[u] = a.part[(size_t)(c0 + u) * a.n + p];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c0 + u < a.nchunk) merge(s, unpack(r[u]));
        }
        if (s.v1 - s.v2 > kGap) {
            a.assign[p] = s.i1;
        } else if (s.v1 - s.v3 > kGap) {
            const int e = atomicAdd(&sN2, 1);
            sP2[e] = p;
            sA2[e] = s.i1;
            sB2[e] = s.i2;
        } else {
            sP3[atomicAdd(&sN3, 1)] = p;
        }
    }
    __syncthreads();
    const int n2 = sN2, n3 = sN3;
    // Two candidates: lanes split the 144 terms, a butterfly sums them.
    for (int e = wave; e < n2; e += KM_FIX / 64) {
        const int q = sP2[e], ia = sA2[e], ib = sB2[e];
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int k = lane + 64 * i;
            if (k < 144) {
                const double x = patch_elem(a, q, k);
                ta = fma(x, a.C64[(size_t)ia * 144 + k], ta);
                tb = fma(x, a.C64[(size_t)ib * 144 + k], tb);
            }
        }
        const double da = wave_sum(ta), db = wave_sum(tb);
        const double mx = fmax(da, db);
        const bool oka = da >= mx - kTie, okb = db >= mx - kTie;
        const int win = (oka && okb) ? min(ia, ib) : (oka ? ia : ib);
        if (lane == 0) a.assign[q] = win;
    }
    // Three or more candidates: up to KM_G3 patches at a time against every
    // centroid.  Thread t takes centroids t, t + KM_FIX, ... from the k-major
    // copy (coalesced), each element serving every patch of the group (FP64
    // FMAs in k order).  Pass 1 finds each patch's largest dot product, pass 2
    // the lowest index within kTie of it; shadowed centroids are skipped.
    for (int g0 = 0; g0 < n3; g0 += KM_G3) {
        const int ng = min(KM_G3, n3 - g0);
        __syncthreads();   // the previous group's rows and slots are consumed
        for (int e = tid; e < KM_G3 * 144; e += KM_FIX) {
            const int j = e / 144, k = e - j * 144;
            sX[j][k] = j < ng ? (double)patch_elem(a, sP3[g0 + j], k) : 0.0;
        }
        __syncthreads();
        double mx[KM_G3];
#pragma unroll
        for (int j = 0; j < KM_G3; ++j) mx[j] = -INFINITY;
        for (int d = tid; d < a.D; d += KM_FIX) {
            if (a.shadow[d]) continue;
            double t[KM_G3];
#pragma unroll
            for (int j = 0; j < KM_G3; ++j) t[j] = 0.0;
            dots_g3(a, d, sX, t);
#pragma unroll
            for (int j = 0; j < KM_G3; ++j) mx[j] = fmax(mx[j], t[j]);
        }
#pragma unroll
        for (int j = 0; j < KM_G3; ++j) {
            double v = mx[j];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
            if (lane == 0) sRed[j][wave] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KM_G3; ++j) {
            double v = sRed[j][0];
            for (int w = 1; w < KM_FIX / 64; ++w) v = fmax(v, sRed[j][w]);
            mx[j] = v;
        }
        int first[KM_G3];
#pragma unroll
        for (int j = 0; j < KM_G3; ++j) first[j] = 0x7fffffff;
        for (int d = tid; d < a.D; d += KM_FIX) {   // ascending: a thread's first hit is its lowest
            if (a.shadow[d]) continue;
            double t[KM_G3];
#pragma unroll
            for (int j = 0; j < KM_G3; ++j) t[j] = 0.0;
            dots_g3(a, d, sX, t);
#pragma unroll
            for (int j = 0; j < KM_G3; ++j)
                if (first[j] == 0x7fffffff && t[j] >= mx[j] - kTie) first[j] = d;
        }
#pragma unroll
        for (int j = 0; j < KM_G3; ++j) {
            int f = first[j];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) f = min(f, __shfl_xor(f, m));
            if (lane == 0) sRedI[j][wave] = f;
        }
        __syncthreads();
        if (tid < ng) {
            int f = sRedI[tid][0];
            for (int w = 1; w < KM_FIX / 64; ++w) f = min(f, sRedI[tid][w]);
            a.assign[sP3[g0 + tid]] = f < a.D ? f : 0;   // no candidate only with non-finite inputs
        }
    }
    if (tid == 0 && (n2 || n3)) {
        atomicAdd(&a.stat[0], n2);
        atomicAdd(&a.stat[1], n3);
    }
}

// Centroid update, pass 1: block (centroid d, patch segment) sums the
// members of d in its segment (each wave a quarter of it, members in order)
// and writes the partial sum of the segment.
__global__ __launch_bounds__(256) void k_km_update(KmArgs a) {
    __shared__ double sPart[4][144];
    const int d = blockIdx.x, seg = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int per_seg = (a.n + a.nsplit - 1) / a.nsplit;
    const int q0 = seg * per_seg, q1 = min(a.n, q0 + per_seg);
    const int per = (q1 - q0 + 3) / 4, p0 = q0 + wave * per, p1 = min(q1, p0 + per);
    double s[3] = {0.0, 0.0, 0.0};
    constexpr int AHEAD = 8;   // assignment loads in flight
    for (int b0 = p0; b0 < p1; b0 += 64 * AHEAD) {
        int av[AHEAD];
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            const int q = b0 + 64 * u + lane;
            av[u] = q < p1 ? a.assign[q] : -1;
        }
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            const int base = b0 + 64 * u;
            unsigned long long m = __ballot(av[u] == d);
            while (m) {   // members in order, four rows' loads in flight
                int j[4];
                int cnt = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    j[w] = m ? __ffsll((long long)m) - 1 : -1;
                    if (m) {
                        m &= m - 1;
                        ++cnt;
                    }
                }
                float x[4][3];
#pragma unroll
                for (int w = 0; w < 4; ++w)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const int k = lane + 64 * i;
                        x[w][i] = (w < cnt && k < 144) ? patch_elem(a, base + j[w], k) : 0.f;
                    }
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    if (w < cnt)
#pragma unroll
                        for (int i = 0; i < 3; ++i) s[i] += (double)x[w][i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = lane + 64 * i;
        if (k < 144) sPart[wave][k] = s[i];
    }
    __syncthreads();
    if (tid < 144)
        a.upd[((size_t)seg * a.D + d) * 144 + tid] =
            ((sPart[0][tid] + sPart[1][tid]) + sPart[2][tid]) + sPart[3][tid];
}

// Pass 2, one wave per centroid: the segments' sums added in order, then the
// rescale to norm 4.  A centroid without members keeps its value.
__global__ __launch_bounds__(64) void k_km_norm(KmArgs a) {
    const int d = blockIdx.x, lane = threadIdx.x;
    double t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = lane + 64 * i;
        double v = 0.0;
        if (k < 144)
            for (int s0 = 0; s0 < a.nsplit; s0 += 4) {   // four segments' loads in flight, added in order
                double r[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    r[u] = s0 + u < a.nsplit ? a.upd[((size_t)(s0 + u) * a.D + d) * 144 + k] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (s0 + u < a.nsplit) v += r[u];
            }
        t[i] = v;
    }
    const double n2 = wave_sum(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    if (!(n2 > 0.0)) return;
    const double sc = 4.0 / sqrt(n2);
    unsigned long long h = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int k = lane + 64 * i;
        if (k < 144) {
            put_centroid(a, d, k, t[i] * sc);
            h ^= elem_hash(t[i] * sc, k);
        }
    }
    h = wave_xor(h);
    if (lane == 0) a.hash[d] = h;
}

}  // namespace

int kmeans_chunks(int D) { return (D + KM_CH - 1) / KM_CH; }

int kmeans_update_splits(int D) {
    const int s = (2048 + D - 1) / D;
    return s < 1 ? 1 : (s > 16 ? 16 : s);
}

hipError_t launch_kmeans(const KmArgs& a, int iters, hipStream_t s) {
    if (a.D < 1 || a.D > DM_MAX_PROTOTYPES || a.D > a.n || a.nchunk != kmeans_chunks(a.D) ||
        a.nsplit != kmeans_update_splits(a.D))
        return hipErrorInvalidValue;
    const bool nt2 = (long)((a.n + 127) / 128) * a.nchunk >= 512;
    const dim3 g_assign((a.n + (nt2 ? 127 : 63)) / (nt2 ? 128 : 64), a.nchunk), g_fix((a.n + KM_FIX - 1) / KM_FIX);
    const dim3 g_shadow((a.D + 3) / 4);
    timing_begin("kmeans_init", 0, s);
    hipLaunchKernelGGL(k_km_init, dim3(a.D), dim3(64), 0, s, a);
    timing_end(s);
    timing_begin("kmeans_shadow", 0, s);
    hipLaunchKernelGGL(k_km_shadow, g_shadow, dim3(256), 0, s, a);
    timing_end(s);
    hipError_t e = hipGetLastError();
    for (int it = 0; it <= iters && e == hipSuccess; ++it) {
        timing_begin("kmeans_assign", 0, s);
        if (nt2)
            hipLaunchKernelGGL(k_km_assign<2>, g_assign, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(k_km_assign<1>, g_assign, dim3(256), 0, s, a);
        timing_end(s);
        timing_begin("kmeans_fix", 0, s);
        hipLaunchKernelGGL(k_km_fix, g_fix, dim3(KM_FIX), 0, s, a);
        timing_end(s);
        if (it < iters) {
            timing_begin("kmeans_update", 0, s);
            hipLaunchKernelGGL(k_km_update, dim3(a.D, a.nsplit), dim3(256), 0, s, a);
            timing_end(s);
            timing_begin("kmeans_norm", 0, s);
            hipLaunchKernelGGL(k_km_norm, dim3(a.D), dim3(64), 0, s, a);
            timing_end(s);
            timing_begin("kmeans_shadow", 0, s);
            hipLaunchKernelGGL(k_km_shadow, g_shadow, dim3(256), 0, s, a);
            timing_end(s);
        }
        e = hipGetLastError();
    }
    return e;
}

}  // namespace dm
