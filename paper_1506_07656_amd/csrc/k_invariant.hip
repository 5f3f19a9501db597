// Scale and rotation invariant matching (Sec. 4.2, Algorithm 2): the
// resampling that makes each run's images, and the reciprocal verification
// (Eq. (16)) over the tables that every run's rectified tuples went into.
#include "dm_group.h"

namespace dm {
namespace {

// One output pixel per thread: the composed map of downsizing and turning,
// in FP64, then bilinear weights; neighbours outside the source count 0.
__global__ __launch_bounds__(256) void k_resample(const float* __restrict__ src, int W, int H, int ld,
                                                  float* __restrict__ dst, int Wr, int Hr, double s, double c,
                                                  double sn, double cinx, double ciny, double coutx, double couty) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= Wr * Hr) return;
    const int v = i / Wr, u = i - v * Wr;
    const double du = (double)u - coutx, dv = (double)v - couty;
    const double x = s * (((c * du - sn * dv) + cinx) + 0.5) - 0.5;
    const double y = s * (((sn * du + c * dv) + ciny) + 0.5) - 0.5;
    const double x0 = floor(x), y0 = floor(y);
    const float fx = (float)(x - x0), fy = (float)(y - y0);
    const int ix = (int)fmax(fmin(x0, 1e9), -1e9), iy = (int)fmax(fmin(y0, 1e9), -1e9);
    float acc = 0.f;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int yy = iy + dy, xx = ix + dx;
            const float w = (dy ? fy : 1.f - fy) * (dx ? fx : 1.f - fx);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) acc += w * src[(size_t)yy * ld + xx];
        }
    dst[i] = acc;
}

// Source cell j of I: BestAt(j) names the target T; the match stands when the
// best tuple of T's cell of I' (BestAt') has the same score and target and
// its source lies in cell j.  Compaction in cell order, as k_finalize.
__global__ __launch_bounds__(1024) void k_finalize_rect(const unsigned long long* __restrict__ best,
                                                        const unsigned long long* __restrict__ cell, RectMap m,
                                                        dm_match* __restrict__ out, int* __restrict__ n_out) {
    __shared__ int wsum[16];
    __shared__ int base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ncell = m.cw1 * ((m.H1o + 3) / 4);
    if (tid == 0) base = 0;
    __syncthreads();
    for (int start = 0; start < ncell; start += 1024) {
        const int j = start + tid;
        int flag = 0;
        dm_match r;
        if (j < ncell) {
            const unsigned long long key = best[j];
            if (key) {
                const uint32_t ti = 0xFFFFFFFFu - (uint32_t)key;
                const int ty = ti / m.W2o, tx = ti - ty * m.W2o;
                const unsigned long long kc = cell[(size_t)(ty >> 2) * m.cw2 + (tx >> 2)];
                const uint32_t lo = 0xFFFFFFFFu - (uint32_t)kc;
                const int pidx = lo >> 4, off = lo & 15;
                const int py = pidx / m.W1o, px = pidx - py * m.W1o;
                flag = (kc >> 32) == (key >> 32) && off == (ty & 3) * 4 + (tx & 3) &&
                       (py >> 2) * m.cw1 + (px >> 2) == j;
                r.x1 = px;
                r.y1 = py;
                r.x2 = tx;
                r.y2 = ty;
                r.score = __uint_as_float((uint32_t)(key >> 32));
            }
        }
        const unsigned long long mask = __ballot(flag);
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wave] = __popcll(mask);
        __syncthreads();
        int o = base;
        for (int w = 0; w < wave; ++w) o += wsum[w];
        if (flag) out[o + rank] = r;
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            base += tot;
        }
        __syncthreads();
    }
    if (tid == 0) *n_out = base;
}

}  // namespace

hipError_t launch_resample(const float* src, int W, int H, int ld, float* dst, int Wr, int Hr, double s, double c,
                           double sn, double cinx, double ciny, double coutx, double couty, hipStream_t st) {
    const int n = Wr * Hr;
    hipLaunchKernelGGL(k_resample, dim3((n + 255) / 256), dim3(256), 0, st, src, W, H, ld, dst, Wr, Hr, s, c, sn,
                       cinx, ciny, coutx, couty);
    return hipGetLastError();
}

hipError_t launch_finalize_rect(const uint64_t* best, const uint64_t* cell, const RectMap& m, dm_match* out,
                                int* n_out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_rect, dim3(1), dim3(1024), 0, s, (const unsigned long long*)best,
                       (const unsigned long long*)cell, m, out, n_out);
    return hipGetLastError();
}

}  // namespace dm
