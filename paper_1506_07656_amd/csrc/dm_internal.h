// Internal declarations shared by the host side (planning, validation,
// launches) and the HIP kernels of libdm.so.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "dm.h"

namespace dm {

// Scale and rotation invariant matching (Sec. 4.2): how one run's atomic
// tuples map back to the input images, and the tables shared by all runs
// (per 4x4 cell of I and of I').  on = 0: plain matching.
struct RectMap {
    int on;
    int W1o, H1o, W2o, H2o, cw1, cw2;     // input images and their cells per row
    double s1, s2, c, sn;                 // scales of I and I', cos and sin of theta
    double cinx, ciny, coutx, couty;      // centres of the downsized I' and of the turned canvas
};

// Rectified source pixel of atomic patch (a, b) of a run: s1 (p + 1/2) - 1/2,
// rounded to the nearest pixel; FP64 in this order, no contraction.
__host__ __device__ inline void rect_source(const RectMap& m, int a, int b, int& px, int& py) {
#pragma clang fp contract(off)
    const double x = m.s1 * ((2.0 + 4.0 * a) + 0.5) - 0.5;
    const double y = m.s1 * ((2.0 + 4.0 * b) + 0.5) - 0.5;
    px = (int)floor(x + 0.5);
    py = (int)floor(y + 0.5);
}

// Rectified target pixel of canvas pixel (u, v): s2 (R_theta((u, v) - c_out)
// + c_in + 1/2) - 1/2, rounded; false if it lies outside I'.
__host__ __device__ inline bool rect_target(const RectMap& m, int u, int v, int& tx, int& ty) {
#pragma clang fp contract(off)
    const double du = (double)u - m.coutx, dv = (double)v - m.couty;
    const double qx = (m.c * du - m.sn * dv) + m.cinx;
    const double qy = (m.sn * du + m.c * dv) + m.ciny;
    const double x = m.s2 * (qx + 0.5) - 0.5, y = m.s2 * (qy + 0.5) - 0.5;
    tx = (int)floor(x + 0.5);
    ty = (int)floor(y + 0.5);
    return tx >= 0 && tx < m.W2o && ty >= 0 && ty < m.H2o;
}

// Geometry of one pair as the kernels see it (passed by value).
// Level l lattice: gx[l] x gy[l] centres; maps of C_l: h[l] x w[l].
struct Geom {
    int W1, H1, W2, H2;
    int lmax;
    int gx[DM_MAX_LEVELS], gy[DM_MAX_LEVELS];
    int h[DM_MAX_LEVELS + 1], w[DM_MAX_LEVELS + 1];
    int vstride;  // bytes per validity table (one per level and axis)
    // Approximate DeepMatching: C'_0 holds nslot0 prototype maps and atomic
    // patch p reads map slot0[p]; null for the exact method (map p).
    const int32_t* slot0;
    int nslot0;
    RectMap rect;   // invariant matching: the run's map back to the input images
    // The descriptors are the library's own with mu > 0 (dm_descriptors: a
    // positive ninth component), so every bottom correlation at a target
    // position inside I' is positive and normal: the bottom kernel's clamp
    // at 0 can go.
    int pos_corr;
    int dmstar;     // entry points at the local maxima of every level (bit 4 of the codes marks them):
                    // 1 = path-sum scores, 2 = start/end-point scores, 0 = every top position
};

// Map index, in the level l-1 buffer, of child lattice index c of a level-l
// parent.
__host__ __device__ inline int child_slot(const Geom& g, int l, int c) {
    return (l == 1 && g.slot0) ? g.slot0[c] : c;
}

// Lattice index, at level l-1, of the child of lattice index `a` at level l
// on the side s in {-1,+1} of one axis (Eq. (5): child centre = parent centre
// + 2^l * s).  Level 0 centres are 2+4a, higher levels 4a.
__host__ __device__ inline int child_index(int l, int a, int s) {
    return l == 1 ? a + ((s - 1) >> 1) : a + s * (1 << (l - 2));
}

// Inverse of child_index: the parent (level l) of child index c (level l-1)
// lying on side s of that parent.
__host__ __device__ inline int parent_index(int l, int c, int s) {
    return l == 1 ? c - ((s - 1) >> 1) : c - s * (1 << (l - 2));
}

// Validity table of level l and axis (0 = x, 1 = y) inside the workspace.
__host__ __device__ inline const uint8_t* vtab(const uint8_t* base, const Geom& g, int l, int axis) {
    return base + (size_t)(2 * l + axis) * g.vstride;
}

// Division by a runtime constant d via a multiply-high: exact for numerators
// e with e * d < 2^32 (all tile and block index ranges here are far below).
struct FastDiv {
    uint32_t d, m;
};
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    f.m = d > 1 ? (uint32_t)((0x100000000ull + d - 1) / d) : 0u;
    return f;
}
__device__ inline uint32_t fdiv(uint32_t e, const FastDiv& f) { return f.d == 1 ? e : __umulhi(e, f.m); }

// Rectification R_lambda of Eq. (11) on a non-negative argument.
__device__ inline float rect_pow(float x, float lam) {
    // hardware log2 / exp2 (v_log_f32, v_exp_f32: about 1 ulp on normal inputs)
    return x > 0.f ? __builtin_amdgcn_exp2f(lam * __builtin_amdgcn_logf(x)) : 0.f;
}
__device__ inline double rect_pow(double x, double lam) {
    return x > 0.0 ? exp2(lam * log2(x)) : 0.0;
}

// Error reporting (thread-local text read back by dm_last_error).
dm_status fail(dm_status s, const char* fmt, ...);
void clear_error();
dm_status check_hip(hipError_t e, const char* what);

// Host planning (dm_plan.cpp).
dm_status plan_pair(const dm_params* prm, int W1, int H1, int W2, int H2, dm_plan_info* out);
dm_status check_params(const dm_params* prm);
dm_status plan_grad(const dm_params* prm, int W1, int H1, int W2, int H2, int recompute, dm_grad_plan* out);
Geom make_geom(const dm_plan_info& pi);

// Descriptor parameters with the Gaussian taps precomputed on the host.
constexpr int kMaxRadius = 6;   // smoothing nu <= 2 (LDS budget of the descriptor kernel)
struct DescParams {
    float scale, slope, mu;
    int r1, r2, r3;
    float g1[2 * kMaxRadius + 1], g2[2 * kMaxRadius + 1], g3[2 * kMaxRadius + 1];
};
DescParams make_desc_params(const dm_params* prm);

// Grouped (batched) stages: each .hip file turns one pair's stage into a job
// record (the kernel's arguments for that pair as a byte image, its block
// count and LDS need); jobs of one kind run together in one persistent launch
// (dm_group.h) through launch_group().
enum JobKind : int {
    JK_DESC = 0,
    JK_VALID,
    JK_CORR_BF16,
    JK_CORR_F32,
    JK_LEVEL_STREAM_VEC,
    JK_LEVEL_STREAM,
    JK_LEVEL_POOL,
    JK_LEVEL_TOP,
    JK_FILL,
    JK_BT,
    JK_BT_STREAM,
    JK_TOP_REDUCE,
    JK_FINALIZE,
    JK_TOP_GRAD,
    JK_BWD_LEVEL,
    JK_BWD_LEVEL_STREAM,
    JK_PATCH_BF16,
    JK_PATCH_F32,
    JK_D2COL_BF16,
    JK_D2COL_F32,
    JK_DD1_BF16,
    JK_DD1_F32,
    JK_TG_BF16,
    JK_TG_F32,
    JK_DD1_REDUCE,
    JK_COL2IM,
    JK_BT_STREAM64,
    JK_LEVEL_NARROW,
    JK_BT_STREAM_BOT,     // the streaming backtracking's bottom level (the key tables), per tile width
    JK_BT_STREAM64_BOT,
    JK_LEVEL_STREAM_VEC8,   // level maps of even width (8-byte child row pieces)
    JK_LEVEL_NARROW8,
    JK_COUNT
};

struct JobRec {
    int kind = -1;
    int blocks = 0;     // virtual blocks of this job
    size_t smem = 0;    // dynamic LDS per block
    std::vector<unsigned char> bytes;
    template <class J>
    void set(int k, int nb, size_t lds, const J& j) {
        kind = k;
        blocks = nb;
        smem = lds;
        bytes.resize(sizeof(J));
        memcpy(bytes.data(), &j, sizeof(J));
    }
};
struct GroupLaunch;
// Per-kind launch parameters: job record size, threads per block, resident
// blocks per CU the kernel allows.
size_t job_size(int kind);
hipError_t launch_group(int kind, const GroupLaunch& gl, hipStream_t s);
hipError_t launch_group_desc(int kind, const GroupLaunch& gl, hipStream_t s);
JobRec desc_job(const float* img, int W, int H, int ld, const DescParams& p, float* out, uint16_t* out_bf16);
hipError_t launch_group_corr(int kind, const GroupLaunch& gl, hipStream_t s);
JobRec corr_job(bool bf16, const void* d1, const void* d2, const Geom& g, float lam, float* cp, uint8_t* code);
hipError_t launch_group_level(int kind, const GroupLaunch& gl, hipStream_t s);
JobRec level_job(int l, const float* prev, const uint8_t* vt, const Geom& g, float lam, float* cp, uint8_t* code,
                 float* top, int tro);
hipError_t launch_group_bt(int kind, const GroupLaunch& gl, hipStream_t s);
JobRec bt_job(int l, const float* cp_prev, const uint8_t* code_prev, const float* u_cur, const uint8_t* code_cur,
              const float* top, const uint8_t* vt, const Geom& g, float* u_prev, uint64_t* best, uint64_t* cell,
              int tr);
JobRec top_reduce_job(const float* top, const Geom& g, uint64_t* best, uint64_t* cell);
JobRec finalize_job(const uint64_t* best, const uint64_t* cell, const Geom& g, dm_match* out, int* n_out);
JobRec fill_job(uint64_t* p, size_t n, uint64_t v);
JobRec valid_job(const Geom& g, uint8_t* vt);
hipError_t launch_group_bwd(int kind, const GroupLaunch& gl, hipStream_t s);
JobRec bwd_level_job(int l, const float* dtop, const float* top, const float* gp_cur, const uint8_t* code_cur,
                     const float* cp_prev, const uint8_t* vt, const Geom& g, float lam, float* gp_prev,
                     bool out16 = false);
JobRec top_grad_job(const float* top, const Geom& g, float* dtop);
hipError_t launch_group_bot(int kind, const GroupLaunch& gl, hipStream_t s);
std::vector<JobRec> bot_jobs(bool bf16, const float* gp, const uint8_t* code, const float* d1, const float* d2,
                             const Geom& g, float* part, float* tbuf, void* dense, float* dd1, float* dd2);

// Approximate DeepMatching: spherical k-means of the atomic patches of I
// (k_kmeans.hip).  d1: FP32 descriptors of I; n = gx0 * gy0 patches; D
// centroids; C64 [D][144]; img / img16: the prototype image (4 x 4D pixels,
// 9 floats / 10 bf16 per pixel; img16 may be null); pv*/pi*: [nchunk][n]
// candidates of the FP32 pass (one 16-byte record per chunk and patch);
// C64T: [144][D] copy of C64; upd: [nsplit][D][144] partial member sums;
// hash[D]: order-independent hash
// of each centroid's FP64 values; shadow[D]: 1 if the centroid equals one of
// lower index (it can never be chosen); stat[2]: patches settled in FP64.
typedef float km_f4 __attribute__((ext_vector_type(4)));
struct KmArgs {
    const float* d1;
    int W1, gx0, n, D, nchunk, nsplit;
    double *C64, *C64T;   // [D][144] and its k-major copy [144][D]
    float* img;
    uint16_t* img16;
    int* assign;
    km_f4* part;
    double* upd;
    unsigned long long* hash;
    int* shadow;
    int* stat;
};
constexpr int KM_CH = 64;   // centroids per chunk of the FP32 pass
int kmeans_chunks(int D);
int kmeans_update_splits(int D);   // patch segments of the centroid update
// Byte offsets inside the k-means scratch region (plan.off_kpart).
inline uint64_t km_align(uint64_t x) { return (x + 255) & ~uint64_t(255); }
inline uint64_t km_upd_off(int D, int n) { return km_align((uint64_t)kmeans_chunks(D) * n * 16); }
inline uint64_t km_hash_off(int D, int n) {
    return km_upd_off(D, n) + km_align((uint64_t)kmeans_update_splits(D) * D * 144 * 8);
}
inline uint64_t km_shadow_off(int D, int n) { return km_hash_off(D, n) + km_align((uint64_t)D * 8); }
inline uint64_t km_c64t_off(int D, int n) { return km_shadow_off(D, n) + km_align((uint64_t)D * 4); }
inline uint64_t km_scratch_bytes(int D, int n) { return km_c64t_off(D, n) + (uint64_t)D * 144 * 8; }
hipError_t launch_kmeans(const KmArgs& a, int iters, hipStream_t s);

// Stages a1..a4 of one pair on descriptors in device memory (dm_api.cpp);
// with rect, a run of invariant matching reducing into rbest / rcell.
// own_desc: d1, d2 (and their BF16 copies when have_bf16) come from the
// library's descriptor kernel.
dm_status run_match(const float* d1, const float* d2, const dm_plan_info& pi, const dm_params* prm, void* ws,
                    bool have_bf16, bool own_desc, dm_match* out, int* n_out, hipStream_t s,
                    const RectMap* rect = nullptr,
                    uint64_t* rbest = nullptr, uint64_t* rcell = nullptr);

// Opt-in stage timing (dm_timing.cpp); calls may nest.
void timing_begin(const char* name, int level, hipStream_t s);
void timing_end(hipStream_t s);
// While suppressed (counted per thread), launches of this thread record no events.
void timing_suppress(bool on);
// dm_match_images on a given workspace (validates everything but clears no error text).
dm_status match_images(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2, int ld2,
                       const dm_params* prm, void* ws, size_t ws_bytes, dm_match* out, int capacity, int* n_out,
                       hipStream_t stream);

// Kernel launchers (each returns the launch status).
hipError_t launch_valid_init(const Geom& g, uint8_t* vt, hipStream_t s);
hipError_t launch_descriptor(const float* img, int W, int H, int ld, const DescParams& p,
                             float* out, uint16_t* out_bf16, hipStream_t s);
hipError_t launch_descriptor_pair(const float* img1, int W1, int H1, int ld1, float* out1, uint16_t* bf1,
                                  const float* img2, int W2, int H2, int ld2, float* out2, uint16_t* bf2,
                                  const DescParams& p, hipStream_t s);
hipError_t launch_to_bf16(const float* d, int n_pix, uint16_t* out, hipStream_t s);
hipError_t launch_corr_pool_f32(const float* d1, const float* d2, const Geom& g, float lam,
                                float* cp, uint8_t* code, hipStream_t s);
hipError_t launch_corr_pool_bf16(const uint16_t* d1, const uint16_t* d2, const Geom& g, float lam,
                                 float* cp, uint8_t* code, hipStream_t s);
template <typename T>
hipError_t launch_corr_top(const T* d1, const T* d2, const Geom& g, T lam, T* top, hipStream_t s);
template <typename T>
hipError_t launch_corr_pool_ref(const T* d1, const T* d2, const Geom& g, T lam, T* cp,
                                uint8_t* code, hipStream_t s);
template <typename T>
hipError_t launch_level(int l, const T* prev, const uint8_t* vt, const Geom& g, T lam, T* cp,
                        uint8_t* code, T* top, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s);
// Marks (bit 4 of the code) the local maxima of the pooled maps C'_l (DM* entry points).
hipError_t launch_mark_entries(int l, const float* cp, uint8_t* code, const uint8_t* vt, const Geom& g,
                               hipStream_t s);
template <typename T>
hipError_t launch_bwd_level(int l, const T* dtop, const T* top, const T* gp_cur, const uint8_t* code_cur,
                            const T* cp_prev, const uint8_t* vt, const Geom& g, T lam, T* gp_prev, hipStream_t s,
                            bool out16 = false);
// mode 0: FP32 MFMA, 1: BF16 MFMA operands with FP32 accumulation (then the pooled gradient gp is
// stored as BF16: the level-1 adjoint writes it with out16), 2: reference kernels (any T)
// dense: scratch of bwd_dense_bytes() for the GEMM operands built from D1 and D2 (modes 0, 1)
template <typename T>
hipError_t launch_bwd_bottom(int mode, const T* gp, const uint8_t* code, const T* d1, const T* d2, const Geom& g,
                             T* part, T* tbuf, void* dense, T* dd1, T* dd2, hipStream_t s);
int bwd_nsplit(const Geom& g);
size_t bwd_dense_bytes(const Geom& g, int precision);
size_t bwd_t_bytes(const Geom& g, int precision);
template <typename T>
hipError_t launch_backtrack(int l, const T* cp_prev, const uint8_t* code_prev, const T* u_cur,
                            const uint8_t* code_cur, const T* top, const uint8_t* vt, const Geom& g,
                            T* u_prev, uint64_t* best, uint64_t* cell, hipStream_t s);
template <typename T>
hipError_t launch_top_reduce(const T* top, const Geom& g, uint64_t* best, uint64_t* cell,
                             hipStream_t s);
hipError_t launch_finalize(const uint64_t* best, const uint64_t* cell, const Geom& g,
                           dm_match* out, int* n_out, hipStream_t s);
// Invariant matching: reciprocal check over the shared tables of all runs.
hipError_t launch_finalize_rect(const uint64_t* best, const uint64_t* cell, const RectMap& m, dm_match* out,
                                int* n_out, hipStream_t s);
// One bilinear resampling (zero outside): canvas pixel (u, v) of dst (Wr x Hr)
// reads src at s (R((u, v) - c_out) + c_in + 1/2) - 1/2, R = [[c, -sn], [sn, c]].
hipError_t launch_resample(const float* src, int W, int H, int ld, float* dst, int Wr, int Hr, double s, double c,
                           double sn, double cinx, double ciny, double coutx, double couty, hipStream_t st);

}  // namespace dm
