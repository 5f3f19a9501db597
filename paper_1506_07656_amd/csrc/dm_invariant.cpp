// Scale and rotation invariant matching (Sec. 4.2, Algorithm 2): plans the
// runs of the (sigma, theta) grid, enqueues them one after the other on the
// caller's stream (each is the plain pipeline on a resampled pair whose
// bottom step maps its tuples back to the input images into tables shared by
// all runs), then one reciprocal verification over those tables.
#include <math.h>
#include <string.h>

#include "dm_internal.h"

namespace dm {
void clear_error();
}  // namespace dm

using namespace dm;

namespace {

// cos and sin of r pi/4: exact table values (0, +-1, and the double nearest
// to sqrt(1/2)), so every run's geometry is reproducible bit for bit.
constexpr double kSqrtHalf = 0.7071067811865476;
constexpr double kCos[8] = {1.0, kSqrtHalf, 0.0, -kSqrtHalf, -1.0, -kSqrtHalf, 0.0, kSqrtHalf};
constexpr double kSin[8] = {0.0, kSqrtHalf, 1.0, kSqrtHalf, 0.0, -kSqrtHalf, -1.0, -kSqrtHalf};

// 2^(|k|/2): a power of two, times sqrt(2) for odd k (exact operations).
double scale_factor(int k) {
    k = k < 0 ? -k : k;
    const double f = (double)(1 << (k / 2));
    return (k & 1) ? f * sqrt(2.0) : f;
}

struct RunGeom {
    int k, r;
    double s1, s2;
    int W1s, H1s;          // I downsized by s1
    int W2s, H2s, Wr, Hr;  // I' downsized by s2, and its turned canvas
    double cinx, ciny, coutx, couty;
};

RunGeom run_geom(int W1, int H1, int W2, int H2, int k, int r) {
#pragma clang fp contract(off)
    RunGeom g;
    g.k = k;
    g.r = r;
    g.s1 = k > 0 ? scale_factor(k) : 1.0;
    g.s2 = k < 0 ? scale_factor(k) : 1.0;
    g.W1s = (int)floor(W1 / g.s1);
    g.H1s = (int)floor(H1 / g.s1);
    g.W2s = (int)floor(W2 / g.s2);
    g.H2s = (int)floor(H2 / g.s2);
    const double c = fabs(kCos[r]), sn = fabs(kSin[r]);
    g.Wr = (int)ceil(g.W2s * c + g.H2s * sn);
    g.Hr = (int)ceil(g.W2s * sn + g.H2s * c);
    g.cinx = (g.W2s - 1) / 2.0;
    g.ciny = (g.H2s - 1) / 2.0;
    g.coutx = (g.Wr - 1) / 2.0;
    g.couty = (g.Hr - 1) / 2.0;
    return g;
}

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

template <typename P>
inline P* at(void* ws, uint64_t off) {
    return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

dm_status plan_invariant(const dm_params* prm, int W1, int H1, int W2, int H2, uint32_t smask, uint32_t rmask,
                         dm_invariant_info* out, RunGeom* runs) {
    if (!out) return fail(DM_ERR_INVALID_ARG, "plan output is null");
    dm_status st = check_params(prm);
    if (st != DM_OK) return st;
    if (prm->precision == DM_FP64) return fail(DM_ERR_UNSUPPORTED, "invariant matching runs in FP32 or BF16");
    if (prm->prototypes) return fail(DM_ERR_UNSUPPORTED, "invariant matching runs the exact method (prototypes = 0)");
    if (prm->entry_points) return fail(DM_ERR_UNSUPPORTED, "invariant matching starts from every top-level position");
    if (!smask || (smask & ~0x1FFu)) return fail(DM_ERR_INVALID_ARG, "scales_mask must be a non-empty subset of 0x1FF");
    if (!rmask || (rmask & ~0xFFu)) return fail(DM_ERR_INVALID_ARG, "rotations_mask must be a non-empty subset of 0xFF");
    if (W1 < 4 || H1 < 4) return fail(DM_ERR_SHAPE, "image 1 is %dx%d; it must hold one 4x4 patch", W1, H1);
    if (W2 < 1 || H2 < 1) return fail(DM_ERR_SHAPE, "image 2 is %dx%d", W2, H2);
    if (W1 > DM_MAX_DIM || H1 > DM_MAX_DIM || W2 > DM_MAX_DIM || H2 > DM_MAX_DIM)
        return fail(DM_ERR_SHAPE, "image sizes above %d are not supported", DM_MAX_DIM);
    memset(out, 0, sizeof(*out));
    uint64_t run_ws = 0, img1 = 0, img2 = 0;
    int n = 0;
    for (int k = -4; k <= 4; ++k) {
        if (!(smask >> (k + 4) & 1u)) continue;
        for (int r = 0; r < 8; ++r) {
            if (!(rmask >> r & 1u)) continue;
            const RunGeom g = run_geom(W1, H1, W2, H2, k, r);
            if (g.W1s < 4 || g.H1s < 4 || g.Wr < 1 || g.Hr < 1) continue;   // no atomic patch: nothing to add
            dm_plan_info pi;
            if ((st = plan_pair(prm, g.W1s, g.H1s, g.Wr, g.Hr, &pi)) != DM_OK) return st;
            out->run_k[n] = k;
            out->run_r[n] = r;
            out->run_W1[n] = g.W1s;
            out->run_H1[n] = g.H1s;
            out->run_W2[n] = g.Wr;
            out->run_H2[n] = g.Hr;
            if (runs) runs[n] = g;
            ++n;
            run_ws = run_ws > pi.workspace_bytes ? run_ws : pi.workspace_bytes;
            img1 = img1 > (uint64_t)g.W1s * g.H1s ? img1 : (uint64_t)g.W1s * g.H1s;
            img2 = img2 > (uint64_t)g.Wr * g.Hr ? img2 : (uint64_t)g.Wr * g.Hr;
        }
    }
    out->n_runs = n;
    out->max_matches = ((W1 + 3) / 4) * ((H1 + 3) / 4);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    out->off_best = take((uint64_t)out->max_matches * 8);
    out->off_cell = take((uint64_t)((W2 + 3) / 4) * ((H2 + 3) / 4) * 8);
    out->off_img1 = take(img1 * 4);
    out->off_img2 = take(img2 * 4);
    out->off_run = take(run_ws);
    out->workspace_bytes = off;
    return DM_OK;
}

// Launches one stage (bracketed by timing events when timing is enabled).
#define DM_LAUNCH(name, level, expr)                 \
    do {                                             \
        timing_begin((name), (level), s);            \
        const hipError_t e_ = (expr);                \
        timing_end(s);                               \
        const dm_status st_ = check_hip(e_, (name)); \
        if (st_ != DM_OK) return st_;                \
    } while (0)

}  // namespace

extern "C" {

dm_status dm_plan_invariant(const dm_params* prm, int W1, int H1, int W2, int H2, uint32_t scales_mask,
                            uint32_t rotations_mask, dm_invariant_info* out) {
    clear_error();
    return plan_invariant(prm, W1, H1, W2, H2, scales_mask, rotations_mask, out, nullptr);
}

dm_status dm_match_invariant(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2,
                             int ld2, const dm_params* prm, uint32_t scales_mask, uint32_t rotations_mask,
                             void* ws, size_t ws_bytes, dm_match* out, int capacity, int* n_out,
                             hipStream_t stream) {
    clear_error();
    dm_invariant_info info;
    RunGeom runs[DM_INV_MAX_RUNS];
    dm_status st = plan_invariant(prm, W1, H1, W2, H2, scales_mask, rotations_mask, &info, runs);
    if (st != DM_OK) return st;
    if (!img1 || !img2) return fail(DM_ERR_INVALID_ARG, "image pointer is null");
    if (ld1 < W1 || ld2 < W2) return fail(DM_ERR_SHAPE, "leading dimension below the width");
    if (!ws) return fail(DM_ERR_INVALID_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < info.workspace_bytes)
        return fail(DM_ERR_WORKSPACE, "workspace holds %zu bytes, the plan needs %llu", ws_bytes,
                    (unsigned long long)info.workspace_bytes);
    if (!out || !n_out) return fail(DM_ERR_INVALID_ARG, "output pointer is null");
    if (capacity < info.max_matches)
        return fail(DM_ERR_CAPACITY, "capacity %d is below the %d matches one call can return", capacity,
                    info.max_matches);
    hipStream_t s = stream;
    uint64_t* best = at<uint64_t>(ws, info.off_best);
    uint64_t* cell = at<uint64_t>(ws, info.off_cell);
    float* i1 = at<float>(ws, info.off_img1);
    float* i2 = at<float>(ws, info.off_img2);
    void* rws = at<void>(ws, info.off_run);
    DM_LAUNCH("fill", -1, launch_fill_u64(best, (size_t)info.max_matches, 0, s));
    DM_LAUNCH("fill", -1, launch_fill_u64(cell, (size_t)((W2 + 3) / 4) * ((H2 + 3) / 4), 0, s));
    const DescParams dp = make_desc_params(prm);
    const bool bf = prm->precision == DM_BF16;
    RectMap m;
    memset(&m, 0, sizeof(m));
    m.on = 1;
    m.W1o = W1;
    m.H1o = H1;
    m.W2o = W2;
    m.H2o = H2;
    m.cw1 = (W1 + 3) / 4;
    m.cw2 = (W2 + 3) / 4;
    for (int j = 0; j < info.n_runs; ++j) {
        const RunGeom& g = runs[j];
        dm_plan_info pi;
        if ((st = plan_pair(prm, g.W1s, g.H1s, g.Wr, g.Hr, &pi)) != DM_OK) return st;
        DM_LAUNCH("resample", -1,
                  launch_resample(img1, W1, H1, ld1, i1, g.W1s, g.H1s, g.s1, 1.0, 0.0, (g.W1s - 1) / 2.0,
                                  (g.H1s - 1) / 2.0, (g.W1s - 1) / 2.0, (g.H1s - 1) / 2.0, s));
        DM_LAUNCH("resample", -1,
                  launch_resample(img2, W2, H2, ld2, i2, g.Wr, g.Hr, g.s2, kCos[g.r], kSin[g.r], g.cinx, g.ciny,
                                  g.coutx, g.couty, s));
        float* d1 = at<float>(rws, pi.off_desc1);
        float* d2 = at<float>(rws, pi.off_desc2);
        DM_LAUNCH("descriptor", -1,
                  launch_descriptor_pair(i1, g.W1s, g.H1s, g.W1s, d1, bf ? at<uint16_t>(rws, pi.off_bf1) : nullptr, i2,
                                         g.Wr, g.Hr, g.Wr, d2, bf ? at<uint16_t>(rws, pi.off_bf2) : nullptr, dp, s));
        m.s1 = g.s1;
        m.s2 = g.s2;
        m.c = kCos[g.r];
        m.sn = kSin[g.r];
        m.cinx = g.cinx;
        m.ciny = g.ciny;
        m.coutx = g.coutx;
        m.couty = g.couty;
        if ((st = run_match(d1, d2, pi, prm, rws, bf, true, nullptr, nullptr, s, &m, best, cell)) != DM_OK)
            return st;
    }
    DM_LAUNCH("finalize", -1, launch_finalize_rect(best, cell, m, out, n_out, s));
    return DM_OK;
}

}  // extern "C"
