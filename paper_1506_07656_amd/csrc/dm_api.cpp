// C-ABI entry points of libdm.so (declared in include/dm.h).  Every call
// validates its arguments on the host, then enqueues the stages of the hot
// path on the caller's stream; nothing here allocates device memory.
#include <string.h>

#include <type_traits>

#include "dm_internal.h"

namespace dm {
const char* last_error_text();
}  // namespace dm

using namespace dm;

namespace {

template <typename P>
inline P* at(void* ws, uint64_t off) {
    return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

// Launches one stage (bracketed by timing events when timing is enabled).
#define DM_LAUNCH(name, level, expr)                                  \
    do {                                                              \
        timing_begin((name), (level), s);                             \
        const hipError_t e_ = (expr);                                 \
        timing_end(s);                                                \
        const dm_status st_ = check_hip(e_, (name));                  \
        if (st_ != DM_OK) return st_;                                 \
    } while (0)

}  // namespace

// Stages a1..a4 on descriptors d1, d2 (float32) already in device memory.
// With rect (a run of invariant matching), the bottom step reduces into the
// shared tables rbest / rcell through the run's map and nothing is
// finalised here.
dm_status dm::run_match(const float* d1, const float* d2, const dm_plan_info& pi, const dm_params* prm, void* ws,
                        bool have_bf16, bool own_desc, dm_match* out, int* n_out, hipStream_t s,
                        const RectMap* rect,
                        uint64_t* rbest, uint64_t* rcell) {
    Geom g = make_geom(pi);
    // The library's own descriptors with mu > 0: the ninth component is at
    // least mu / sqrt(8 + mu^2), and every window of a target position inside
    // I' holds that position's own pixel, so A_0 >= (mu^2 / (8 + mu^2)) / 16
    // > 2^-126 for mu >= 1e-6.
    g.pos_corr = own_desc && prm->mu >= 1e-6f;
    if (rect) g.rect = *rect;
    const float lam = prm->lambda;
    uint8_t* vt = at<uint8_t>(ws, pi.off_valid);
    DM_LAUNCH("valid_init", -1, launch_valid_init(g, vt, s));
    float* top = at<float>(ws, pi.off_top);
    auto cp = [&](int l) { return at<float>(ws, pi.off_cp[l]); };
    auto code = [&](int l) { return at<uint8_t>(ws, pi.off_code[l]); };
    auto u = [&](int l) { return at<float>(ws, pi.off_u[l]); };
    // a1: bottom correlation + rectification + pooled level 0.
    if (pi.prototypes > 0) {
        // Approximate DeepMatching (Sec. 4.1): the D prototype maps, computed
        // by the bottom kernels on the prototype image (one row of D atomic
        // patches); level 1 and the bottom backtracking read patch p's map
        // through the assignment.
        const int D = pi.prototypes;
        const int na = pi.n_atomic;
        KmArgs km;
        km.d1 = d1;
        km.W1 = pi.W1;
        km.gx0 = pi.gx[0];
        km.n = na;
        km.D = D;
        km.nchunk = pi.kmeans_chunks;
        km.nsplit = kmeans_update_splits(D);
        km.C64 = at<double>(ws, pi.off_protos);
        km.img = at<float>(ws, pi.off_proto_img);
        km.img16 = prm->precision == DM_BF16 ? at<uint16_t>(ws, pi.off_proto_bf) : nullptr;
        km.assign = at<int>(ws, pi.off_assign);
        km.part = at<km_f4>(ws, pi.off_kpart);
        km.upd = at<double>(ws, pi.off_kpart + km_upd_off(D, na));
        km.hash = at<unsigned long long>(ws, pi.off_kpart + km_hash_off(D, na));
        km.shadow = at<int>(ws, pi.off_kpart + km_shadow_off(D, na));
        km.C64T = at<double>(ws, pi.off_kpart + km_c64t_off(D, na));
        km.stat = at<int>(ws, pi.off_kstat);
        const dm_status st = check_hip(launch_kmeans(km, prm->kmeans_iters, s), "kmeans");
        if (st != DM_OK) return st;
        Geom gp = g;   // the prototype image: 4 x 4D pixels, D atomic patches in one row
        gp.W1 = 4 * D;
        gp.H1 = 4;
        gp.gx[0] = D;
        gp.gy[0] = 1;
        if (prm->precision == DM_BF16) {
            uint16_t* b2 = at<uint16_t>(ws, pi.off_bf2);
            if (!have_bf16) DM_LAUNCH("to_bf16", -1, launch_to_bf16(d2, pi.W2 * pi.H2, b2, s));
            DM_LAUNCH("corr_pool_bf16", 0, launch_corr_pool_bf16(km.img16, b2, gp, lam, cp(0), code(0), s));
        } else {
            DM_LAUNCH("corr_pool_f32", 0, launch_corr_pool_f32(km.img, d2, gp, lam, cp(0), code(0), s));
        }
        g.slot0 = km.assign;
        g.nslot0 = D;
    } else if (pi.lmax == 0) {
        DM_LAUNCH("corr_top", 0, launch_corr_top<float>(d1, d2, g, lam, top, s));
    } else if (prm->precision == DM_BF16) {
        uint16_t* b1 = at<uint16_t>(ws, pi.off_bf1);
        uint16_t* b2 = at<uint16_t>(ws, pi.off_bf2);
        if (!have_bf16) {
            DM_LAUNCH("to_bf16", -1, launch_to_bf16(d1, pi.W1 * pi.H1, b1, s));
            DM_LAUNCH("to_bf16", -1, launch_to_bf16(d2, pi.W2 * pi.H2, b2, s));
        }
        DM_LAUNCH("corr_pool_bf16", 0, launch_corr_pool_bf16(b1, b2, g, lam, cp(0), code(0), s));
    } else {
        DM_LAUNCH("corr_pool_f32", 0, launch_corr_pool_f32(d1, d2, g, lam, cp(0), code(0), s));
    }
    // a2: levels 1..lmax.
    for (int l = 1; l <= pi.lmax; ++l)
        DM_LAUNCH("level", l, launch_level<float>(l, cp(l - 1), vt, g, lam, l < pi.lmax ? cp(l) : nullptr,
                                                  l < pi.lmax ? code(l) : nullptr, top, s));
    // DM* entry points: the local maxima of every pooled level (the top's are
    // tested during its backtracking step).
    if (prm->entry_points == DM_ENTRIES_LOCAL_MAXIMA) {
        g.dmstar = prm->scoring == DM_SCORE_START_END ? 2 : 1;
        for (int l = 0; l < pi.lmax; ++l) DM_LAUNCH("mark_entries", l, launch_mark_entries(l, cp(l), code(l), vt, g, s));
    }
    // a3 + a4: backtracking, bottom reduction, reciprocal check, compaction.
    uint64_t* best = rect ? rbest : at<uint64_t>(ws, pi.off_best);
    uint64_t* cell = rect ? rcell : at<uint64_t>(ws, pi.off_cell);
    if (!rect) {
        DM_LAUNCH("fill", -1, launch_fill_u64(best, (size_t)pi.n_atomic, 0, s));
        DM_LAUNCH("fill", -1, launch_fill_u64(cell, (size_t)((pi.H2 + 3) / 4) * ((pi.W2 + 3) / 4), 0, s));
    }
    if (pi.lmax == 0) {
        DM_LAUNCH("top_reduce", 0, launch_top_reduce<float>(top, g, best, cell, s));
    } else {
        for (int l = pi.lmax; l >= 1; --l)
            DM_LAUNCH("backtrack", l,
                      launch_backtrack<float>(l, cp(l - 1), code(l - 1), l < pi.lmax ? u(l) : nullptr,
                                              l < pi.lmax ? code(l) : nullptr, top, vt, g,
                                              l >= 2 ? u(l - 1) : nullptr, best, cell, s));
    }
    if (!rect) DM_LAUNCH("finalize", -1, launch_finalize(best, cell, g, out, n_out, s));
    return DM_OK;
}

namespace {

dm_status check_ws(const dm_plan_info& pi, void* ws, size_t ws_bytes) {
    if (!ws) return fail(DM_ERR_INVALID_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < pi.workspace_bytes)
        return fail(DM_ERR_WORKSPACE, "workspace holds %zu bytes, the plan needs %llu", ws_bytes,
                    (unsigned long long)pi.workspace_bytes);
    return DM_OK;
}

dm_status check_out(const dm_plan_info& pi, dm_match* out, int capacity, int* n_out) {
    if (!out || !n_out) return fail(DM_ERR_INVALID_ARG, "output pointer is null");
    if (capacity < pi.max_matches)
        return fail(DM_ERR_CAPACITY, "capacity %d is below the %d matches one call can return", capacity,
                    pi.max_matches);
    return DM_OK;
}

dm_status check_grad_bufs(const dm_grad_plan& gp, const void* d1, const void* d2, const void* saved,
                          size_t saved_bytes, void* scratch, size_t scratch_bytes) {
    if (!d1 || !d2) return fail(DM_ERR_INVALID_ARG, "descriptor pointer is null");
    if (!saved || !scratch) return fail(DM_ERR_INVALID_ARG, "saved or scratch buffer is null");
    if ((reinterpret_cast<uintptr_t>(saved) | reinterpret_cast<uintptr_t>(scratch)) & 255)
        return fail(DM_ERR_INVALID_ARG, "saved and scratch buffers must be 256-byte aligned");
    if (saved_bytes < gp.saved_bytes || scratch_bytes < gp.scratch_bytes)
        return fail(DM_ERR_WORKSPACE, "buffers hold %zu / %zu bytes, the plan needs %llu / %llu", saved_bytes,
                    scratch_bytes, (unsigned long long)gp.saved_bytes, (unsigned long long)gp.scratch_bytes);
    return DM_OK;
}

// Pointers of the grad layout.
template <typename T>
struct GradBufs {
    const dm_grad_plan& gp;
    void* saved;
    void* scratch;
    T* cp(int l) const { return at<T>(gp.cp_in_saved[l] ? saved : scratch, gp.off_cp[l]); }
    uint8_t* code(int l) const { return at<uint8_t>(gp.cp_in_saved[l] ? saved : scratch, gp.off_code[l]); }
    T* top() const { return at<T>(saved, gp.off_top); }
    uint8_t* vt() const { return at<uint8_t>(scratch, gp.off_valid); }
    T* gbuf(int i) const { return at<T>(scratch, gp.off_g[i]); }
};

// Levels first..last of the pyramid (C'_l and codes, or C_top at lmax).
template <typename T>
dm_status run_levels(const GradBufs<T>& B, const Geom& g, int first, int last, T lam, hipStream_t s) {
    for (int l = first; l <= last; ++l)
        DM_LAUNCH("level", l, launch_level<T>(l, B.cp(l - 1), B.vt(), g, lam, l < g.lmax ? B.cp(l) : nullptr,
                                              l < g.lmax ? B.code(l) : nullptr, B.top(), s));
    return DM_OK;
}

template <typename T>
dm_status grad_forward(const T* d1, const T* d2, const dm_grad_plan& gp, const dm_params* prm, void* saved,
                       void* scratch, hipStream_t s) {
    const Geom g = make_geom(gp.geom);
    const GradBufs<T> B{gp, saved, scratch};
    const T lam = (T)prm->lambda;
    DM_LAUNCH("valid_init", -1, launch_valid_init(g, B.vt(), s));
    if constexpr (std::is_same<T, double>::value) {
        DM_LAUNCH("corr_pool_ref", 0, launch_corr_pool_ref<double>(d1, d2, g, lam, B.cp(0), B.code(0), s));
    } else if (prm->precision == DM_BF16) {
        uint16_t* b1 = at<uint16_t>(scratch, gp.off_bf1);
        uint16_t* b2 = at<uint16_t>(scratch, gp.off_bf2);
        DM_LAUNCH("to_bf16", -1, launch_to_bf16(d1, g.W1 * g.H1, b1, s));
        DM_LAUNCH("to_bf16", -1, launch_to_bf16(d2, g.W2 * g.H2, b2, s));
        DM_LAUNCH("corr_pool_bf16", 0, launch_corr_pool_bf16(b1, b2, g, lam, B.cp(0), B.code(0), s));
    } else {
        DM_LAUNCH("corr_pool_f32", 0, launch_corr_pool_f32(d1, d2, g, lam, B.cp(0), B.code(0), s));
    }
    return run_levels<T>(B, g, 1, g.lmax, lam, s);
}

template <typename T>
dm_status grad_backward(const T* d1, const T* d2, const dm_grad_plan& gp, const dm_params* prm, void* saved,
                        const T* dtop, T* dd1, T* dd2, void* scratch, hipStream_t s) {
    const Geom g = make_geom(gp.geom);
    const GradBufs<T> B{gp, saved, scratch};
    const T lam = (T)prm->lambda;
    DM_LAUNCH("valid_init", -1, launch_valid_init(g, B.vt(), s));
    if (gp.recompute && g.lmax > 1) {
        const dm_status st = run_levels<T>(B, g, 1, g.lmax - 1, lam, s);
        if (st != DM_OK) return st;
    }
    const int mode = std::is_same<T, double>::value ? 2 : (prm->precision == DM_BF16 ? 1 : 0);
    const bool g16 = mode == 1;   // the BF16 bottom reads the level-1 gradient as BF16
    for (int l = g.lmax; l >= 1; --l) {
        const T* gcur = l < g.lmax ? B.gbuf(l & 1) : nullptr;
        DM_LAUNCH("bwd_level", l,
                  launch_bwd_level<T>(l, dtop, B.top(), gcur, l < g.lmax ? B.code(l) : nullptr, B.cp(l - 1), B.vt(),
                                      g, lam, B.gbuf((l - 1) & 1), s, l == 1 && g16));
    }
    DM_LAUNCH("bwd_bottom", 0,
              launch_bwd_bottom<T>(mode, B.gbuf(0), B.code(0), d1, d2, g, at<T>(scratch, gp.off_part),
                                   at<T>(scratch, gp.off_t), at<void>(scratch, gp.off_dense), dd1, dd2, s));
    return DM_OK;
}

}  // namespace

// dm_match_images on the workspace ws (validated here; the caller has
// cleared the error text).
dm_status dm::match_images(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2, int ld2,
                           const dm_params* prm, void* ws, size_t ws_bytes, dm_match* out, int capacity,
                           int* n_out, hipStream_t stream) {
    dm_plan_info pi;
    dm_status st = plan_pair(prm, W1, H1, W2, H2, &pi);
    if (st != DM_OK) return st;
    if (!img1 || !img2) return fail(DM_ERR_INVALID_ARG, "image pointer is null");
    if (ld1 < W1 || ld2 < W2) return fail(DM_ERR_SHAPE, "leading dimension below the width");
    if ((st = check_ws(pi, ws, ws_bytes)) != DM_OK) return st;
    if ((st = check_out(pi, out, capacity, n_out)) != DM_OK) return st;
    if (prm->precision == DM_FP64) return fail(DM_ERR_UNSUPPORTED, "matching runs in FP32 or BF16");
    const DescParams dp = make_desc_params(prm);
    float* d1 = at<float>(ws, pi.off_desc1);
    float* d2 = at<float>(ws, pi.off_desc2);
    const bool bf = prm->precision == DM_BF16;
    hipStream_t s = stream;
    DM_LAUNCH("descriptor", -1,
              launch_descriptor_pair(img1, W1, H1, ld1, d1, bf ? at<uint16_t>(ws, pi.off_bf1) : nullptr, img2, W2, H2,
                                     ld2, d2, bf ? at<uint16_t>(ws, pi.off_bf2) : nullptr, dp, s));
    return run_match(d1, d2, pi, prm, ws, bf, true, out, n_out, stream);
}

extern "C" {

dm_status dm_plan_grad(const dm_params* prm, int W1, int H1, int W2, int H2, int recompute, dm_grad_plan* out) {
    clear_error();
    return plan_grad(prm, W1, H1, W2, H2, recompute, out);
}

dm_status dm_pyramid_forward(const void* d1, int W1, int H1, const void* d2, int W2, int H2, const dm_params* prm,
                             int recompute, void* saved, size_t saved_bytes, void* scratch, size_t scratch_bytes,
                             hipStream_t stream) {
    clear_error();
    dm_grad_plan gp;
    dm_status st = plan_grad(prm, W1, H1, W2, H2, recompute, &gp);
    if (st != DM_OK) return st;
    if ((st = check_grad_bufs(gp, d1, d2, saved, saved_bytes, scratch, scratch_bytes)) != DM_OK) return st;
    if (prm->precision == DM_FP64)
        return grad_forward<double>((const double*)d1, (const double*)d2, gp, prm, saved, scratch, stream);
    return grad_forward<float>((const float*)d1, (const float*)d2, gp, prm, saved, scratch, stream);
}

dm_status dm_pyramid_backward(const void* d1, int W1, int H1, const void* d2, int W2, int H2, const dm_params* prm,
                              int recompute, const void* saved, size_t saved_bytes, const void* dc_top, void* dd1,
                              void* dd2, void* scratch, size_t scratch_bytes, hipStream_t stream) {
    clear_error();
    dm_grad_plan gp;
    dm_status st = plan_grad(prm, W1, H1, W2, H2, recompute, &gp);
    if (st != DM_OK) return st;
    if ((st = check_grad_bufs(gp, d1, d2, saved, saved_bytes, scratch, scratch_bytes)) != DM_OK) return st;
    if (!dc_top || !dd1 || !dd2) return fail(DM_ERR_INVALID_ARG, "gradient pointer is null");
    void* sv = const_cast<void*>(saved);
    if (prm->precision == DM_FP64)
        return grad_backward<double>((const double*)d1, (const double*)d2, gp, prm, sv, (const double*)dc_top,
                                     (double*)dd1, (double*)dd2, scratch, stream);
    return grad_backward<float>((const float*)d1, (const float*)d2, gp, prm, sv, (const float*)dc_top, (float*)dd1,
                                (float*)dd2, scratch, stream);
}

dm_status dm_default_params(dm_params* p) {
    clear_error();
    if (!p) return fail(DM_ERR_INVALID_ARG, "params is null");
    memset(p, 0, sizeof(*p));
    p->nu1 = 0.f;
    p->nu2 = 1.f;
    p->nu3 = 1.f;
    p->sigmoid_slope = 0.2f;
    p->mu = 0.1f;
    p->intensity_scale = 255.f;
    p->lambda = 1.4f;
    p->max_patch = 0;
    p->precision = DM_FP32;
    p->prototypes = 0;
    p->kmeans_iters = 10;
    return DM_OK;
}

dm_status dm_plan(const dm_params* prm, int W1, int H1, int W2, int H2, dm_plan_info* out) {
    clear_error();
    return plan_pair(prm, W1, H1, W2, H2, out);
}

dm_status dm_descriptors(const float* img, int W, int H, int ld, const dm_params* prm, float* desc,
                         hipStream_t stream) {
    clear_error();
    dm_status st = check_params(prm);
    if (st != DM_OK) return st;
    if (!img || !desc) return fail(DM_ERR_INVALID_ARG, "image or descriptor pointer is null");
    if (W < 1 || H < 1 || W > DM_MAX_DIM || H > DM_MAX_DIM) return fail(DM_ERR_SHAPE, "image is %dx%d", W, H);
    if (ld < W) return fail(DM_ERR_SHAPE, "leading dimension %d < width %d", ld, W);
    const DescParams dp = make_desc_params(prm);
    hipStream_t s = stream;
    DM_LAUNCH("descriptor", -1, launch_descriptor(img, W, H, ld, dp, desc, nullptr, s));
    return DM_OK;
}

dm_status dm_match_descriptors(const void* d1, int W1, int H1, const void* d2, int W2, int H2,
                               const dm_params* prm, void* ws, size_t ws_bytes, dm_match* out, int capacity,
                               int* n_out, hipStream_t stream) {
    clear_error();
    dm_plan_info pi;
    dm_status st = plan_pair(prm, W1, H1, W2, H2, &pi);
    if (st != DM_OK) return st;
    if (!d1 || !d2) return fail(DM_ERR_INVALID_ARG, "descriptor pointer is null");
    if ((st = check_ws(pi, ws, ws_bytes)) != DM_OK) return st;
    if ((st = check_out(pi, out, capacity, n_out)) != DM_OK) return st;
    if (prm->precision == DM_FP64) return fail(DM_ERR_UNSUPPORTED, "matching runs in FP32 or BF16");
    return run_match((const float*)d1, (const float*)d2, pi, prm, ws, false, false, out, n_out, stream);
}

dm_status dm_match_images(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2, int ld2,
                          const dm_params* prm, void* ws, size_t ws_bytes, dm_match* out, int capacity,
                          int* n_out, hipStream_t stream) {
    clear_error();
    return match_images(img1, W1, H1, ld1, img2, W2, H2, ld2, prm, ws, ws_bytes, out, capacity, n_out, stream);
}

const char* dm_status_string(dm_status s) {
    switch (s) {
        case DM_OK: return "ok";
        case DM_ERR_INVALID_ARG: return "invalid argument";
        case DM_ERR_SHAPE: return "unsupported shape";
        case DM_ERR_WORKSPACE: return "workspace too small";
        case DM_ERR_CAPACITY: return "output capacity too small";
        case DM_ERR_UNSUPPORTED: return "unsupported mode";
        case DM_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* dm_last_error(void) { return last_error_text(); }

const char* dm_version(void) { return "dm-mi355x 0.1"; }

}  // extern "C"
