// Host-side planning of one image pair: parameter checks, pyramid levels
// (Algorithm 1 with the boundary rule of Sec. 3.2), patch grids (Eq. (7)),
// map sizes and the workspace layout.  Touches no device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "dm_internal.h"

namespace {
thread_local char g_err[512] = "";

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
}  // namespace

namespace dm {

dm_status fail(dm_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

dm_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return DM_OK;
    return fail(DM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

dm_status check_params(const dm_params* p) {
    if (!p) return fail(DM_ERR_INVALID_ARG, "params is null");
    const float vals[7] = {p->nu1, p->nu2, p->nu3, p->sigmoid_slope, p->mu, p->intensity_scale, p->lambda};
    for (float v : vals)
        if (!isfinite(v)) return fail(DM_ERR_INVALID_ARG, "non-finite parameter");
    const float nus[3] = {p->nu1, p->nu2, p->nu3};
    for (float nu : nus)
        if (nu < 0.f || ceilf(3.f * nu) > (float)kMaxRadius)
            return fail(DM_ERR_INVALID_ARG, "smoothing nu must be in [0, %d]", kMaxRadius / 3);
    if (p->sigmoid_slope <= 0.f) return fail(DM_ERR_INVALID_ARG, "sigmoid_slope must be > 0");
    if (p->mu < 0.f) return fail(DM_ERR_INVALID_ARG, "mu must be >= 0");
    if (p->intensity_scale <= 0.f) return fail(DM_ERR_INVALID_ARG, "intensity_scale must be > 0");
    if (p->lambda < 1.f || p->lambda > 8.f) return fail(DM_ERR_INVALID_ARG, "lambda must be in [1, 8]");
    if (p->max_patch != 0 &&
        (p->max_patch < 4 || (p->max_patch & (p->max_patch - 1)) || p->max_patch > (4 << (DM_MAX_LEVELS - 1))))
        return fail(DM_ERR_INVALID_ARG, "max_patch must be 0 or a power of two in [4, %d]", 4 << (DM_MAX_LEVELS - 1));
    if (p->precision < DM_FP32 || p->precision > DM_FP64) return fail(DM_ERR_INVALID_ARG, "unknown precision");
    if (p->prototypes < 0 || p->prototypes > DM_MAX_PROTOTYPES)
        return fail(DM_ERR_INVALID_ARG, "prototypes must be in [0, %d]", DM_MAX_PROTOTYPES);
    if (p->kmeans_iters < 0 || p->kmeans_iters > 1000)
        return fail(DM_ERR_INVALID_ARG, "kmeans_iters must be in [0, 1000]");
    if (p->entry_points != DM_ENTRIES_TOP && p->entry_points != DM_ENTRIES_LOCAL_MAXIMA)
        return fail(DM_ERR_INVALID_ARG, "entry_points must be DM_ENTRIES_TOP or DM_ENTRIES_LOCAL_MAXIMA");
    if (p->scoring != DM_SCORE_PATH_SUM && p->scoring != DM_SCORE_START_END)
        return fail(DM_ERR_INVALID_ARG, "scoring must be DM_SCORE_PATH_SUM or DM_SCORE_START_END");
    if (p->scoring == DM_SCORE_START_END && p->entry_points != DM_ENTRIES_LOCAL_MAXIMA)
        return fail(DM_ERR_UNSUPPORTED, "start/end-point scoring comes with the local-maxima entry points");
    for (int r : p->reserved)
        if (r != 0) return fail(DM_ERR_INVALID_ARG, "reserved fields must be 0");
    return DM_OK;
}

// 1-D validity of the lattice of each level along one axis: an index exists
// when one of its two children (Eq. (5)) exists at the level below.
static void axis_validity(int g0, int gl, int lmax, std::vector<std::vector<uint8_t>>& v) {
    v.assign(lmax + 1, {});
    v[0].assign(g0, 1);
    for (int l = 1; l <= lmax; ++l) {
        const int nprev = l == 1 ? g0 : gl;
        v[l].assign(gl, 0);
        for (int a = 0; a < gl; ++a)
            for (int s = -1; s <= 1; s += 2) {
                const int c = child_index(l, a, s);
                if (c >= 0 && c < nprev && v[l - 1][c]) v[l][a] = 1;
            }
    }
}

dm_status plan_pair(const dm_params* prm, int W1, int H1, int W2, int H2, dm_plan_info* out) {
    if (!out) return fail(DM_ERR_INVALID_ARG, "plan output is null");
    dm_status st = check_params(prm);
    if (st != DM_OK) return st;
    if (W1 < 4 || H1 < 4) return fail(DM_ERR_SHAPE, "image 1 is %dx%d; it must hold one 4x4 patch", W1, H1);
    if (W2 < 1 || H2 < 1) return fail(DM_ERR_SHAPE, "image 2 is %dx%d", W2, H2);
    if (W1 > DM_MAX_DIM || H1 > DM_MAX_DIM || W2 > DM_MAX_DIM || H2 > DM_MAX_DIM)
        return fail(DM_ERR_SHAPE, "image sizes above %d are not supported", DM_MAX_DIM);
    memset(out, 0, sizeof(*out));
    out->W1 = W1;
    out->H1 = H1;
    out->W2 = W2;
    out->H2 = H2;
    out->precision = prm->precision;

    // Pyramid top: Algorithm 1's loop bound or the explicit N_max.
    int N = 4;
    if (prm->max_patch) {
        N = prm->max_patch;
    } else {
        while (N < (W1 > H1 ? W1 : H1)) N *= 2;
    }
    int lmax = 0;
    while ((4 << lmax) < N) ++lmax;
    if (lmax > DM_MAX_LEVELS - 1) lmax = DM_MAX_LEVELS - 1;

    const int g0x = W1 / 4, g0y = H1 / 4;
    const int glx = (W1 - 1) / 4 + 1, gly = (H1 - 1) / 4 + 1;
    std::vector<std::vector<uint8_t>> vx, vy;
    axis_validity(g0x, glx, lmax, vx);
    axis_validity(g0y, gly, lmax, vy);
    // Cap at the last level whose grid is non-empty.
    for (;;) {
        int cx = 0, cy = 0;
        for (uint8_t b : vx[lmax]) cx += b;
        for (uint8_t b : vy[lmax]) cy += b;
        if ((cx && cy) || lmax == 0) break;
        --lmax;
    }
    const int D = prm->prototypes;
    if (D > 0) {
        if (prm->precision == DM_FP64)
            return fail(DM_ERR_UNSUPPORTED, "approximate matching runs in FP32 or BF16");
        if (D > g0x * g0y)
            return fail(DM_ERR_INVALID_ARG, "%d prototypes for %d atomic patches", D, g0x * g0y);
        if (lmax == 0)
            return fail(DM_ERR_UNSUPPORTED, "approximate matching needs a pooled level (N_max >= 8)");
    }
    if (prm->entry_points == DM_ENTRIES_LOCAL_MAXIMA) {
        if (D > 0) return fail(DM_ERR_UNSUPPORTED, "local-maxima entry points run the exact method (prototypes = 0)");
        if (lmax == 0) return fail(DM_ERR_UNSUPPORTED, "local-maxima entry points need a pooled level (N_max >= 8)");
    }
    out->lmax = lmax;
    out->N_max = 4 << lmax;
    out->n_atomic = g0x * g0y;
    out->max_matches = out->n_atomic;
    for (int l = 0; l <= lmax; ++l) {
        out->gx[l] = l ? glx : g0x;
        out->gy[l] = l ? gly : g0y;
        int cx = 0, cy = 0;
        for (uint8_t b : vx[l]) cx += b;
        for (uint8_t b : vy[l]) cy += b;
        out->n_valid[l] = cx * cy;
    }
    out->h[0] = H2;
    out->w[0] = W2;
    for (int l = 1; l <= lmax + 1; ++l) {
        out->h[l] = (out->h[l - 1] + 1) / 2;
        out->w[l] = (out->w[l - 1] + 1) / 2;
    }

    // Workspace layout.
    const uint64_t es = prm->precision == DM_FP64 ? 8 : 4;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    out->off_misc = take(256);
    out->off_desc1 = take((uint64_t)W1 * H1 * 9 * es);
    out->off_desc2 = take((uint64_t)W2 * H2 * 9 * es);
    if (prm->precision == DM_BF16) {
        out->off_bf1 = take((uint64_t)W1 * H1 * 10 * 2);
        out->off_bf2 = take((uint64_t)W2 * H2 * 10 * 2);
    }
    const int vstride = (int)align256((uint64_t)(glx > gly ? glx : gly));
    out->off_valid = take((uint64_t)(lmax + 1) * 2 * vstride);
    for (int l = 0; l < lmax; ++l) {
        const uint64_t maps = (l == 0 && D > 0) ? (uint64_t)D : (uint64_t)out->gx[l] * out->gy[l];
        const uint64_t n = maps * out->h[l + 1] * out->w[l + 1];
        out->off_cp[l] = take(n * es);
        out->off_code[l] = take(n);
        if (l >= 1) out->off_u[l] = take(n * es);
    }
    out->off_top = take((uint64_t)out->gx[lmax] * out->gy[lmax] * out->h[lmax] * out->w[lmax] * es);
    out->off_best = take((uint64_t)out->n_atomic * 8);
    out->off_cell = take((uint64_t)((H2 + 3) / 4) * ((W2 + 3) / 4) * 8);
    if (D > 0) {
        const uint64_t na = (uint64_t)out->n_atomic;
        out->prototypes = D;
        out->kmeans_chunks = kmeans_chunks(D);
        out->off_protos = take((uint64_t)D * 144 * 8);
        out->off_assign = take(na * 4);
        out->off_kstat = take(2 * 4);
        out->off_proto_img = take((uint64_t)D * 144 * 4);
        if (prm->precision == DM_BF16) out->off_proto_bf = take((uint64_t)D * 160 * 2);
        out->off_kpart = take(km_scratch_bytes(D, (int)na));
    }
    out->workspace_bytes = off;
    return DM_OK;
}

dm_status plan_grad(const dm_params* prm, int W1, int H1, int W2, int H2, int recompute, dm_grad_plan* out) {
    if (!out) return fail(DM_ERR_INVALID_ARG, "plan output is null");
    dm_plan_info pi;
    dm_status st = plan_pair(prm, W1, H1, W2, H2, &pi);
    if (st != DM_OK) return st;
    if (pi.lmax == 0) return fail(DM_ERR_UNSUPPORTED, "the pyramid has a single level; nothing to route a gradient through");
    if (prm->prototypes) return fail(DM_ERR_UNSUPPORTED, "the gradient is that of the exact method (prototypes = 0)");
    if (prm->entry_points) return fail(DM_ERR_UNSUPPORTED, "entry points concern matching, not the gradient");
    // The bottom GEMMs address the pooled gradient of 128 patches from one
    // 32-bit buffer offset.
    if (prm->precision != DM_FP64 && (uint64_t)128 * pi.h[1] * pi.w[1] * 4 >= (uint64_t(1) << 31))
        return fail(DM_ERR_SHAPE, "image 2 is %dx%d; the gradient supports at most %d pooled positions", W2, H2,
                    (1 << 31) / 512 - 1);
    memset(out, 0, sizeof(*out));
    out->geom = pi;
    out->recompute = recompute ? 1 : 0;
    const Geom g = make_geom(pi);
    const bool fp64 = prm->precision == DM_FP64;
    out->nsplit = fp64 ? 1 : bwd_nsplit(g);
    const uint64_t es = fp64 ? 8 : 4;
    uint64_t so = 0, xo = 0;  // saved / scratch cursors
    auto take = [](uint64_t& cur, uint64_t bytes) {
        const uint64_t o = cur;
        cur = align256(cur + bytes);
        return o;
    };
    for (int l = 0; l < pi.lmax; ++l) {
        const uint64_t n = (uint64_t)pi.gx[l] * pi.gy[l] * pi.h[l + 1] * pi.w[l + 1];
        const bool keep = l == 0 || !recompute;
        out->cp_in_saved[l] = keep ? 1 : 0;
        out->off_cp[l] = take(keep ? so : xo, n * es);
        out->off_code[l] = take(keep ? so : xo, n);
    }
    out->off_top = take(so, (uint64_t)pi.gx[pi.lmax] * pi.gy[pi.lmax] * pi.h[pi.lmax] * pi.w[pi.lmax] * es);
    const int glx = (W1 - 1) / 4 + 1, gly = (H1 - 1) / 4 + 1;
    const uint64_t vstride = align256((uint64_t)(glx > gly ? glx : gly));
    out->off_valid = take(xo, (uint64_t)(pi.lmax + 1) * 2 * vstride);
    if (prm->precision == DM_BF16) {
        out->off_bf1 = take(xo, (uint64_t)W1 * H1 * 10 * 2);
        out->off_bf2 = take(xo, (uint64_t)W2 * H2 * 10 * 2);
    }
    // Gradients of the pooled maps C'_l, l < lmax, alternate between two
    // buffers; each holds the largest of them.  Levels above 0 have
    // ceil(W/4) x ceil(H/4) lattice points against floor(W/4) x floor(H/4)
    // at level 0, so with tiny maps a coarser level can be the largest.
    uint64_t ng = 0;
    for (int l = 0; l < pi.lmax; ++l) {
        const uint64_t n = (uint64_t)pi.gx[l] * pi.gy[l] * pi.h[l + 1] * pi.w[l + 1];
        if (n > ng) ng = n;
    }
    out->off_g[0] = take(xo, ng * es);
    out->off_g[1] = take(xo, ng * es);
    out->off_part = take(xo, (uint64_t)out->nsplit * pi.n_atomic * 144 * es);
    out->off_t = take(xo, bwd_t_bytes(g, prm->precision));
    if (!fp64) out->off_dense = take(xo, bwd_dense_bytes(g, prm->precision));
    out->saved_bytes = so;
    out->scratch_bytes = xo;
    return DM_OK;
}

Geom make_geom(const dm_plan_info& pi) {
    Geom g;
    memset(&g, 0, sizeof(g));
    g.W1 = pi.W1;
    g.H1 = pi.H1;
    g.W2 = pi.W2;
    g.H2 = pi.H2;
    g.lmax = pi.lmax;
    for (int l = 0; l <= pi.lmax; ++l) {
        g.gx[l] = pi.gx[l];
        g.gy[l] = pi.gy[l];
    }
    for (int l = 0; l <= pi.lmax + 1 && l <= DM_MAX_LEVELS; ++l) {
        g.h[l] = pi.h[l];
        g.w[l] = pi.w[l];
    }
    const int glx = (pi.W1 - 1) / 4 + 1, gly = (pi.H1 - 1) / 4 + 1;
    g.vstride = (int)align256((uint64_t)(glx > gly ? glx : gly));
    return g;
}

DescParams make_desc_params(const dm_params* prm) {
    DescParams d;
    memset(&d, 0, sizeof(d));
    d.scale = prm->intensity_scale;
    d.slope = prm->sigmoid_slope;
    d.mu = prm->mu;
    const float nus[3] = {prm->nu1, prm->nu2, prm->nu3};
    int* rs[3] = {&d.r1, &d.r2, &d.r3};
    float* gs[3] = {d.g1, d.g2, d.g3};
    for (int k = 0; k < 3; ++k) {
        const double s = nus[k];
        if (s <= 0) {
            *rs[k] = 0;
            gs[k][0] = 1.f;
            continue;
        }
        const int r = (int)ceil(3.0 * s);
        double tot = 0;
        double tmp[2 * kMaxRadius + 1];
        for (int t = -r; t <= r; ++t) tot += (tmp[t + r] = exp(-(double)t * t / (2.0 * s * s)));
        for (int t = 0; t <= 2 * r; ++t) gs[k][t] = (float)(tmp[t] / tot);
        *rs[k] = r;
    }
    return d;
}

const char* last_error_text() { return g_err; }
void clear_error() { g_err[0] = 0; }

}  // namespace dm
