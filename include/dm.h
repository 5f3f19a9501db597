/*
 * dm.h -- C ABI of the MI355X DeepMatching library (libdm.so).
 *
 * The library computes the hot path of DeepMatching (Revaud, Weinzaepfel,
 * Harchaoui, Schmid, "DeepMatching: Hierarchical Deformable Dense Matching",
 * IJCV 2016): per-pixel descriptors (Sec. 3.2, "Pixel descriptor"), the
 * bottom-up multi-level correlation pyramid (Sec. 3.2, Eqs. (3)-(12),
 * Algorithm 1) and the top-down backtracking with merging and reciprocal
 * verification (Sec. 3.3, Eqs. (13)-(16)).  Given two images I (W x H) and
 * I' (W' x H') it returns quasi-dense correspondences (p, p', s).
 *
 * Conventions shared by every entry point:
 *  - Pixels are 0-based, x to the right, y down.  Images are row-major
 *    float32 grey values in [0, 1] with a leading dimension `ld` (>= W,
 *    in elements).  Descriptors are float32, H x W x 9, channel innermost.
 *  - Every buffer is owned by the caller.  Pointers named *_host are host
 *    memory; all others are device memory of the current HIP device.  The
 *    library allocates no device memory: scratch space comes from the caller
 *    as a workspace whose size dm_plan() reports.
 *  - Calls that take a stream enqueue their work on it and return without
 *    waiting; results are ready once the stream has reached that point.
 *    Arguments are validated on the host before anything is enqueued; on an
 *    error nothing is enqueued and dm_last_error() describes the problem.
 *  - Output capacity: the match count n_out lives in device memory and is
 *    written by the enqueued work, so an insufficient capacity is reported
 *    by DM_ERR_CAPACITY alone (nothing is enqueued, n_out is untouched); the
 *    required capacity is plan.max_matches (info.max_matches for invariant
 *    matching), known on the host from dm_plan / dm_plan_invariant before
 *    any call, and dm_last_error() repeats it.
 *  - The library keeps no state between calls other than the thread-local
 *    error text, the per-stage timing records (when enabled), for
 *    dm_match_batch one cached batch schedule per workspace (job tables,
 *    chosen tile shapes and, with DM_BATCH_GRAPH, an instantiated HIP graph),
 *    dropped by dm_batch_release, for dm_deepflow with DM_FLOW_GRAPH one
 *    instantiated graph per workspace, dropped by dm_flow_release, and the
 *    static per-device scratch array of dm_match_images_noalloc.  Calls on different streams with different
 *    workspaces may run concurrently; two calls sharing a workspace must be
 *    ordered.
 */
#ifndef DM_H
#define DM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DM_MAX_LEVELS 16   /* level index l < 16, patch size N = 4 * 2^l   */
#define DM_MAX_DIM 8192    /* largest supported image width or height      */
#define DM_MAX_PROTOTYPES 4096  /* largest prototype dictionary (Sec. 4.1) */

typedef enum {
    DM_OK = 0,
    DM_ERR_INVALID_ARG = -1,   /* null pointer, bad parameter value          */
    DM_ERR_SHAPE = -2,         /* image smaller than one atomic patch, too big */
    DM_ERR_WORKSPACE = -3,     /* workspace smaller than dm_plan() reports   */
    DM_ERR_CAPACITY = -4,      /* output smaller than plan.max_matches       */
    DM_ERR_UNSUPPORTED = -5,   /* precision or mode not available for a call */
    DM_ERR_HIP = -6            /* a HIP runtime call failed                  */
} dm_status;

typedef enum {
    DM_FP32 = 0,   /* bottom correlation on FP32 MFMA, pyramid FP32          */
    DM_BF16 = 1,   /* bottom correlation on BF16 MFMA with FP32 accumulation */
    DM_FP64 = 2    /* every stage in FP64 (gradient checks)                  */
} dm_precision;

/* Method parameters.  Descriptor (Sec. 3.2 "Pixel descriptor", values of
 * Sec. 5.2.1 for uncompressed images): Gaussian smoothing with standard
 * deviation nu1 before the gradient (0 = none), nu2 on the 8 oriented
 * gradient maps, nu3 after the sigmoid 2/(1+exp(-sigmoid_slope x))-1, the
 * ninth component mu, intensities multiplied by intensity_scale.
 * Rectification exponent lambda (Eq. (11)).  max_patch: pyramid top N_max
 * (power of two >= 4), 0 = the loop bound of Algorithm 1 (N < max(W, H));
 * either way capped at the last level whose patch grid is non-empty.
 *
 * Approximate DeepMatching (Sec. 4.1), matching calls only: with
 * prototypes = D > 0 the atomic patches of I are clustered by spherical
 * k-means into D prototypes (centroids kept at the norm 4 of a patch vector,
 * i.e. its 16 unit pixel descriptors in (dy, dx, channel) order), and each
 * patch takes the bottom map C'_0 of its nearest prototype, so the bottom
 * correlation computes and stores D maps instead of one per patch.
 * Centroid d starts as atomic patch floor((2d+1) n / (2D)) of the n patches
 * in raster order; kmeans_iters rounds of assignment (largest dot product;
 * within 1e-11 of the largest, the lowest index) and update (sum of the
 * members rescaled to norm 4; no members: unchanged), then a final
 * assignment.  Decisions are those of an FP64 evaluation.  1 <= D <=
 * min(n, DM_MAX_PROTOTYPES); D = 0 is the exact method. */
typedef struct {
    float nu1, nu2, nu3, sigmoid_slope, mu, intensity_scale, lambda;
    int32_t max_patch;
    int32_t precision;          /* dm_precision */
    int32_t prototypes;         /* D of approximate DeepMatching, 0 = exact     */
    int32_t kmeans_iters;       /* k-means rounds (prototypes > 0), 0..1000     */
    int32_t entry_points;       /* DM_ENTRIES_TOP or DM_ENTRIES_LOCAL_MAXIMA    */
    int32_t scoring;            /* DM_SCORE_PATH_SUM or DM_SCORE_START_END      */
    int32_t reserved[3];        /* must be 0 */
} dm_params;

/* Entry points of the backtracking (Sec. 3.3, "Merging correspondences").
 * DM_ENTRIES_TOP: every position of every top-level map (the method of the
 * paper).  DM_ENTRIES_LOCAL_MAXIMA: the earlier scheme compared in Sec. 5
 * (Table 1, "DM*"), here with the current path-sum scores: the local maxima
 * of the maps of every level start backtracking paths.  The maps are C_top
 * and the pooled C'_l below it (a pooled cell stands for the position it was
 * pooled from, with its value as the entry's score); a local maximum is
 * positive, not below any of its 3 x 3 neighbours inside the map and above
 * those before it in raster order (one per plateau).  Tuples from above and
 * entries merge by max at equal (N, p, p').  Matching entry points only
 * (dm_match_images / dm_match_descriptors), exact method, N_max >= 8; in the
 * workspace, bit 4 of a code (off_code[l]) then marks the entries of C'_l. */
#define DM_ENTRIES_TOP 0
#define DM_ENTRIES_LOCAL_MAXIMA 1

/* Scores of the atomic correspondences.  DM_SCORE_PATH_SUM: the sum of the
 * correlation values along the whole backtracking path (Eq. (14), the
 * method of the paper).  DM_SCORE_START_END: the earlier scheme of Table 1
 * (Sec. 5), which scored a correspondence from the values at the start and
 * the end of its path only: here the entry's value plus the atomic value
 * C'_0 the path ends on (an entry at the bottom level counts its value
 * once), equal (N, p, p') merging by max as before.  Table 1 pairs it with
 * the local-maxima entry points, and so does this library:
 * DM_SCORE_START_END requires entry_points = DM_ENTRIES_LOCAL_MAXIMA
 * (DM_ERR_UNSUPPORTED otherwise). */
#define DM_SCORE_PATH_SUM 0
#define DM_SCORE_START_END 1

/* One correspondence: atomic patch centre p = (x1, y1) in I, pixel
 * p' = (x2, y2) in I', score s = the top-level value plus the pooled child
 * values along the backtracking path (Eq. (14)); with DM_SCORE_START_END the
 * entry's value plus the atomic value at the path's end. */
typedef struct {
    int32_t x1, y1, x2, y2;
    float score;
} dm_match;

/* Geometry and workspace layout of one image pair.  Level l has patches on
 * a lattice of gx[l] x gy[l] candidate centres ((2+4a, 2+4b) at l = 0,
 * (4a, 4b) above), of which n_valid[l] exist (Eq. (7) with the boundary rule
 * of Sec. 3.2); its correlation maps C_l have h[l] x w[l] entries, with
 * h[0] = H', w[0] = W', h[l+1] = ceil(h[l]/2).
 *
 * Workspace contents after a match call (byte offsets from the workspace
 * base, all 256-byte aligned):
 *   off_cp[l]   l < lmax: pooled maps C'_l, float32 [gy][gx][h[l+1]][w[l+1]]
 *               (entries of non-existing patches are undefined)
 *   off_code[l] l < lmax: argmax codes of C'_l, uint8, same shape, value
 *               3(m_y+1)+(m_x+1) of the first maximum (Eq. (9))
 *   off_top     C_lmax, float32 [gy][gx][h[lmax]][w[lmax]]
 *   off_u[l]    1 <= l < lmax: best backtracking score reaching each pooled
 *               node of level l, float32, shape of C'_l, -inf if unreached
 *   off_desc1/2 descriptors of I and I' (dm_match_images), float32 HWC
 *   off_best    per atomic patch: packed best tuple (uint64)
 *   off_cell    per 4x4 target cell: packed best tuple (uint64)
 * With prototypes = D > 0, off_cp[0] / off_code[0] hold the D prototype maps
 * [D][h[1]][w[1]] (patch p's map is that of prototype assign[p]) and
 *   off_protos  the prototypes, float64 [D][144], (dy, dx, channel) order
 *   off_assign  prototype of each atomic patch, int32 [gy[0]][gx[0]]
 *   off_kstat   int32 [2]: assignments settled in FP64 over all k-means
 *               rounds (between two candidates; over every centroid)
 */
typedef struct {
    int32_t W1, H1, W2, H2;
    int32_t lmax;              /* top level index; N_max = 4 << lmax        */
    int32_t N_max;
    int32_t n_atomic;          /* |G_4| = floor(W/4) * floor(H/4)            */
    int32_t max_matches;       /* sufficient output capacity (= n_atomic)    */
    int32_t precision;
    int32_t gx[DM_MAX_LEVELS], gy[DM_MAX_LEVELS], n_valid[DM_MAX_LEVELS];
    int32_t h[DM_MAX_LEVELS + 1], w[DM_MAX_LEVELS + 1];
    uint64_t off_cp[DM_MAX_LEVELS], off_code[DM_MAX_LEVELS], off_u[DM_MAX_LEVELS];
    uint64_t off_top, off_desc1, off_desc2, off_bf1, off_bf2, off_valid;
    uint64_t off_best, off_cell, off_misc;
    int32_t prototypes;        /* D (0: exact method)                         */
    int32_t kmeans_chunks;     /* centroid chunks of the k-means FP32 pass     */
    uint64_t off_protos, off_assign, off_kstat;
    uint64_t off_proto_img, off_proto_bf, off_kpart;   /* k-means scratch     */
    uint64_t workspace_bytes;
} dm_plan_info;

/* Fills *p with the defaults: nu1=0, nu2=nu3=1, sigmoid_slope=0.2, mu=0.1,
 * intensity_scale=255, lambda=1.4, max_patch=0, precision=DM_FP32,
 * prototypes=0 (exact), kmeans_iters=10.
 * Host only.  Errors: DM_ERR_INVALID_ARG if p is null. */
dm_status dm_default_params(dm_params* p);

/* Plans the pyramid of an I (W1 x H1) / I' (W2 x H2) pair: levels, patch
 * grids, map sizes (Algorithm 1 with the boundary rule of Sec. 3.2) and the
 * workspace layout, written to *out.  Host only; touches no device.
 * Errors: DM_ERR_INVALID_ARG (null pointer, parameter out of range,
 * max_patch not a power of two >= 4, prototypes above the number of atomic
 * patches), DM_ERR_SHAPE (W1 or H1 < 4, W2 or H2 < 1, any size above
 * DM_MAX_DIM), DM_ERR_UNSUPPORTED (prototypes with DM_FP64 or with a
 * single-level pyramid). */
dm_status dm_plan(const dm_params* prm, int W1, int H1, int W2, int H2, dm_plan_info* out);

/* Per-pixel descriptors of one image (Sec. 3.2, "Pixel descriptor"):
 * img is W x H float32 with leading dimension ld; desc receives H x W x 9
 * float32 (unit l2 norm, non-negative).  Errors: DM_ERR_INVALID_ARG,
 * DM_ERR_SHAPE (W or H < 1 or > DM_MAX_DIM, ld < W), DM_ERR_HIP. */
dm_status dm_descriptors(const float* img, int W, int H, int ld, const dm_params* prm,
                         float* desc, hipStream_t stream);

/* Matches two descriptor fields (d1: H1 x W1 x 9, d2: H2 x W2 x 9, float32;
 * float64 when prm->precision == DM_FP64): bottom correlation (Eq. (4)),
 * pyramid levels (Eq. (12)), backtracking from every top-level entry with
 * merging (Eq. (15)) and reciprocal verification (Eq. (16)).  Writes the
 * matches, sorted by (y1, x1), to out[0 .. *n_out) and their count to the
 * DEVICE int n_out.  At most one match per atomic patch, so capacity >=
 * plan.max_matches is always enough.  ws must hold plan.workspace_bytes
 * bytes (256-byte aligned); it keeps the pyramid afterwards (see
 * dm_plan_info).  Errors: DM_ERR_INVALID_ARG, DM_ERR_SHAPE,
 * DM_ERR_WORKSPACE, DM_ERR_CAPACITY (capacity < plan.max_matches),
 * DM_ERR_UNSUPPORTED, DM_ERR_HIP. */
dm_status dm_match_descriptors(const void* d1, int W1, int H1, const void* d2, int W2, int H2,
                               const dm_params* prm, void* ws, size_t ws_bytes,
                               dm_match* out, int capacity, int* n_out, hipStream_t stream);

/* dm_descriptors on both images (into the workspace), then
 * dm_match_descriptors.  Same outputs and errors; FP64 is not available on
 * this entry point (DM_ERR_UNSUPPORTED). */
dm_status dm_match_images(const float* img1, int W1, int H1, int ld1,
                          const float* img2, int W2, int H2, int ld2,
                          const dm_params* prm, void* ws, size_t ws_bytes,
                          dm_match* out, int capacity, int* n_out, hipStream_t stream);

/* dm_match_images for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The workspace is a static device array of
 * DM_NOALLOC_MAX_BYTES that every GPU the library runs on holds from the
 * load of the library's code until the process ends; the call allocates
 * nothing (no hipMalloc, no events: per-stage timing records nothing for
 * it).  The caller still passes the images and the outputs (as
 * dm_match_images).  Every call on a GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other host threads) race; the
 * array keeps the last call's pyramid.  Errors: those of dm_match_images,
 * and DM_ERR_WORKSPACE when plan.workspace_bytes exceeds
 * DM_NOALLOC_MAX_BYTES (pairs up to about 192 x 144). */
#define DM_NOALLOC_MAX_BYTES ((size_t)128 << 20)
dm_status dm_match_images_noalloc(const float* img1, int W1, int H1, int ld1,
                                  const float* img2, int W2, int H2, int ld2,
                                  const dm_params* prm, dm_match* out, int capacity, int* n_out,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Scale and rotation invariant matching (Sec. 4.2, Algorithm 2).
 *
 * DeepMatching runs on every selected version of the pair: sigma = k/2 for
 * the set bits k + 4 of scales_mask (k in -4..4; I is downsized by
 * max(1, 2^sigma), I' by max(1, 2^-sigma)) and theta = r pi/4 for the set
 * bits r of rotations_mask (r in 0..7; I' is rotated by -theta).  A
 * downsized or rotated image is one bilinear resampling of the input
 * (pixel centres aligned, zero outside; the rotated image is the bounding
 * box of the turned one).  Every run's raw atomic correspondences
 * (Eq. (15)) are mapped back to the input images, P = s1 (p + 1/2) - 1/2
 * and T = s2 (R_theta (p' - c_out) + c_in + 1/2) - 1/2 in FP64 rounded to
 * the nearest pixel (tuples whose T leaves I' are dropped), and one
 * reciprocal verification (Eq. (16)) runs over their union with the fixed
 * 4x4 cells of P in I and of T in I'.  At most one match per source cell,
 * in row-major order of the source cells; max_matches = ceil(W1/4) *
 * ceil(H1/4).  The paper's grid is scales_mask = 0x1FF, rotations_mask =
 * 0xFF (72 runs); scales_mask = 0x10, rotations_mask = 1 is the plain
 * method.  Runs go one after the other on the stream, reusing the
 * workspace.  Precisions DM_FP32 and DM_BF16; prototypes must be 0.
 * --------------------------------------------------------------------------- */
#define DM_INV_MAX_RUNS 72

typedef struct {
    int32_t n_runs;            /* runs with at least one atomic patch         */
    int32_t max_matches;       /* ceil(W1/4) * ceil(H1/4)                       */
    int32_t run_k[DM_INV_MAX_RUNS], run_r[DM_INV_MAX_RUNS];   /* sigma = k/2, theta = r pi/4 */
    int32_t run_W1[DM_INV_MAX_RUNS], run_H1[DM_INV_MAX_RUNS]; /* downsized I                 */
    int32_t run_W2[DM_INV_MAX_RUNS], run_H2[DM_INV_MAX_RUNS]; /* downsized, turned I'        */
    uint64_t off_best, off_cell, off_img1, off_img2, off_run;  /* workspace layout            */
    uint64_t workspace_bytes;
} dm_invariant_info;

/* Plans the runs of an invariant match (host only).  Errors: those of
 * dm_plan for any run, DM_ERR_INVALID_ARG (empty or out-of-range masks),
 * DM_ERR_UNSUPPORTED (DM_FP64, prototypes != 0). */
dm_status dm_plan_invariant(const dm_params* prm, int W1, int H1, int W2, int H2, uint32_t scales_mask,
                            uint32_t rotations_mask, dm_invariant_info* out);

/* Invariant matches of two images (device buffers, as dm_match_images).
 * Writes the matches to out[0 .. *n_out) and their count to the DEVICE int
 * n_out.  Errors: those of dm_plan_invariant, DM_ERR_WORKSPACE,
 * DM_ERR_CAPACITY (capacity < info.max_matches), DM_ERR_HIP. */
dm_status dm_match_invariant(const float* img1, int W1, int H1, int ld1, const float* img2, int W2, int H2,
                             int ld2, const dm_params* prm, uint32_t scales_mask, uint32_t rotations_mask,
                             void* ws, size_t ws_bytes, dm_match* out, int capacity, int* n_out,
                             hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Gradient of a loss on the top-level maps (no counterpart in the paper).
 *
 * dm_pyramid_forward computes the pyramid of two descriptor fields (Eqs.
 * (3)-(12), Algorithm 1) and keeps what the backward needs in the caller's
 * `saved` buffer: C'_0 and its argmax codes, C_top, and (unless recompute
 * is set) C'_l and codes of every coarser level.  dm_pyramid_backward takes
 * dL/dC_top and returns dL/dD1 and dL/dD2 through the hand-written adjoints of
 * rectification, the shifted average over existing children, the max-pool
 * routed to the stored argmax, and the bottom correlation; with recompute set
 * it first recomputes the coarse levels from C'_0 into scratch.
 * Precision: DM_FP32 (FP32 MFMA GEMMs), DM_BF16 (BF16 operands, FP32
 * accumulation and pyramid) or DM_FP64 (every stage in FP64, direct
 * kernels; meant for finite-difference checks on small inputs).
 * --------------------------------------------------------------------------- */
typedef struct {
    dm_plan_info geom;         /* levels and map sizes (its offsets belong to the match calls) */
    int32_t recompute;
    int32_t nsplit;            /* position splits of the dD1 contraction */
    uint64_t saved_bytes;      /* size of `saved` */
    uint64_t scratch_bytes;    /* size of `scratch` */
    /* Byte offsets of C'_l, codes_l (l < lmax) and C_top: in `saved` when the
     * matching *_in_saved flag is 1, else in `scratch`. */
    uint64_t off_cp[DM_MAX_LEVELS], off_code[DM_MAX_LEVELS];
    int32_t cp_in_saved[DM_MAX_LEVELS];
    uint64_t off_top;          /* in `saved` */
    uint64_t off_valid, off_bf1, off_bf2, off_g[2], off_part, off_t;  /* in `scratch` */
    uint64_t off_dense;        /* in `scratch`: operands of the bottom GEMMs (D2 im2col, D1 patches) */
} dm_grad_plan;

/* Plans dm_pyramid_forward / dm_pyramid_backward for a pair of sizes.
 * Host only.  Errors as dm_plan; DM_ERR_UNSUPPORTED if the pyramid has a
 * single level (N_max = 4: no pooled level to route through) or
 * prototypes != 0 (the gradient is that of the exact method). */
dm_status dm_plan_grad(const dm_params* prm, int W1, int H1, int W2, int H2, int recompute, dm_grad_plan* out);

/* Forward pyramid of descriptor fields d1 (H1 x W1 x 9) and d2 (H2 x W2 x 9),
 * float32 (float64 when prm->precision == DM_FP64).  C_top, [gy][gx][h][w]
 * of the top level (maps of non-existing lattice points are zeros), is left
 * in `saved` at plan.off_top.  Errors: DM_ERR_INVALID_ARG, DM_ERR_SHAPE,
 * DM_ERR_WORKSPACE (either buffer too small), DM_ERR_UNSUPPORTED, DM_ERR_HIP. */
dm_status dm_pyramid_forward(const void* d1, int W1, int H1, const void* d2, int W2, int H2,
                             const dm_params* prm, int recompute, void* saved, size_t saved_bytes,
                             void* scratch, size_t scratch_bytes, hipStream_t stream);

/* Backward of the pyramid left in `saved` by dm_pyramid_forward with the
 * same inputs and parameters: dc_top = dL/dC_top (layout of C_top; entries of
 * non-existing patches are ignored) -> dd1 (H1 x W1 x 9) and dd2 (H2 x W2 x
 * 9), overwritten; pixels outside every atomic patch get 0 in dd1.
 * Deterministic.  Errors as dm_pyramid_forward. */
dm_status dm_pyramid_backward(const void* d1, int W1, int H1, const void* d2, int W2, int H2,
                              const dm_params* prm, int recompute, const void* saved, size_t saved_bytes,
                              const void* dc_top, void* dd1, void* dd2, void* scratch, size_t scratch_bytes,
                              hipStream_t stream);

/* ------------------------------------------------------------------ batches
 * Many image pairs of uneven sizes in one call (a throughput extension: the
 * method itself is defined per pair, Sec. 3, and its per-patch loops are
 * independent, Algorithm 2).  Each pair goes through exactly the stages of
 * dm_match_images, with the same kernels and the same arithmetic, so its
 * matches are identical to those of a dm_match_images call with its images;
 * but every stage runs as ONE persistent grouped launch covering all pairs
 * (a fixed grid of resident blocks walks a table of (pair, tile) work items),
 * so small pairs and the small upper levels fill the GPU together.
 *
 * flags:
 *  DM_BATCH_BWD       also the gradient of the loss L = sum over top-level
 *                     patches P of max_q C_top(P, q) (the top map's first
 *                     maximum takes the gradient) with respect to both
 *                     descriptor fields, into pair.dd1 / pair.dd2; the same
 *                     kernels as dm_pyramid_backward with recompute = 0.
 *  DM_BATCH_GRAPH     capture the whole sequence of launches in a HIP graph on
 *                     the first call and replay it on later calls with the
 *                     same arguments (stream must not be the null stream).
 *  DM_BATCH_AUTOTUNE  on the first call, time candidate tile shapes (band
 *                     heights of the streaming level and backtracking
 *                     kernels, resident blocks per CU of each grouped launch)
 *                     on this batch and keep the fastest (dm_batch_tiles_get).
 *                     Tuned tiles persist in a JSON file, the path in the
 *                     environment variable DM_TILE_CACHE (default
 *                     $HOME/.cache/dm_mi355x/tiles.json; set to "" to turn
 *                     the file off), keyed by precision, direction and a size
 *                     bucket (pair count, largest target width and height,
 *                     total pixels, each rounded up to a power of two); a
 *                     batch whose key is there takes those tiles untimed.
 *                     A file that cannot be read or written is ignored.
 * The schedule (job tables in the workspace, tiles, graph) is cached per
 * workspace and rebuilt when any argument changes.  Precisions DM_FP32 and
 * DM_BF16; every pair needs at least one pooled level (N_max >= 8). */
#define DM_MAX_BATCH 256
#define DM_BATCH_BWD 1
#define DM_BATCH_GRAPH 2
#define DM_BATCH_AUTOTUNE 4

typedef struct {
    const float* img1;   /* I: W1 x H1, leading dimension ld1 (device)      */
    int32_t W1, H1, ld1;
    const float* img2;   /* I': W2 x H2, leading dimension ld2 (device)     */
    int32_t W2, H2, ld2;
    float* dd1;          /* DM_BATCH_BWD: dL/dD1, H1 x W1 x 9 (device)      */
    float* dd2;          /* DM_BATCH_BWD: dL/dD2, H2 x W2 x 9 (device)      */
} dm_pair;

typedef struct {
    int32_t n_pairs;
    int32_t n_launches;                  /* grouped launches per call        */
    int32_t max_matches[DM_MAX_BATCH];   /* per pair (= dm_plan max_matches) */
    int32_t lmax[DM_MAX_BATCH];          /* per pair pyramid top level       */
    uint64_t workspace_bytes;
} dm_batch_info;

typedef struct {
    int32_t level_rows;          /* pooled rows per band, streaming level kernel  */
    int32_t bt_rows;             /* rows per band, streaming backtracking kernel  */
    int32_t blocks_per_cu[32];   /* resident blocks per CU, per grouped kernel kind */
    int32_t tuned;               /* 0 defaults, 1 tuned on this batch, 2 read from the tile cache */
    float tuned_ms;              /* time of the batch with them when tuned        */
} dm_batch_tiles;

/* Sizes of a batch of n pairs (1 <= n <= DM_MAX_BATCH).  Host only; reads
 * the sizes in pairs[] only.  Errors: DM_ERR_INVALID_ARG, DM_ERR_SHAPE,
 * DM_ERR_UNSUPPORTED (FP64, prototypes != 0, or a pair without a pooled
 * level). */
dm_status dm_plan_batch(int n, const dm_pair* pairs, const dm_params* prm, int flags, dm_batch_info* out);

/* Matches of every pair: pair k writes its matches (sorted by (y1, x1)) to
 * out + out_offsets_host[k] and their number to n_out[k] (device).  The
 * caller sizes out so that pair k has max_matches[k] entries from its offset
 * on; offsets must leave that room (checked).  ws (256-byte aligned) must hold
 * info.workspace_bytes and is owned by the batch schedule between calls with
 * the same arguments.  Errors: those of dm_plan_batch, DM_ERR_WORKSPACE,
 * DM_ERR_CAPACITY (overlapping output ranges), DM_ERR_HIP. */
dm_status dm_match_batch(int n, const dm_pair* pairs, const dm_params* prm, int flags, void* ws, size_t ws_bytes,
                         dm_match* out, const int32_t* out_offsets_host, int32_t* n_out, hipStream_t stream);

/* Tile shapes of the schedule cached for workspace ws (host).  Errors:
 * DM_ERR_INVALID_ARG if no schedule is cached for ws. */
dm_status dm_batch_tiles_get(const void* ws, dm_batch_tiles* out);

/* Drops the schedule (and graph) cached for workspace ws; call before freeing
 * or reusing ws for other data.  Errors: none. */
dm_status dm_batch_release(const void* ws);

/* ---------------------------------------------------------------- DeepFlow
 * Variational refinement of a flow field w = (u, v) from I to I' with
 * DeepMatching's matches as its matching term (Sec. 4.3, Eqs. (17)-(19)):
 * E(w) = int E_D + alpha(x) E_S + beta c phi Psi(|w - w'|^2), with E_D the
 * normalised colour (weight delta) and gradient (weight gamma) constancy
 * terms, E_S = Psi(|grad u|^2 + |grad v|^2), alpha(x) = exp(-kappa
 * |grad I|), Psi(s^2) = sqrt(s^2 + eps^2).  Solved coarse to fine (factor
 * eta, down to a smaller side of min_size) with incremental warping,
 * n_fixed fixed-point iterations per level and n_sor red-black SOR sweeps
 * (relaxation omega) per fixed point; beta^k = beta (k / k_max)^b at level k
 * (0 = finest).  phi = sqrt(lam_scale lambda_min) / (sigma_M sqrt(2 pi))
 * exp(-Delta / (2 sigma_M)) per match.  Images are grayscale in [0, 1],
 * smoothed by a Gaussian of standard deviation sigma.  The library's
 * readings of what the paper leaves open are listed in k_deepflow.hip. */
#define DM_FLOW_MAX_LEVELS 128

typedef struct {
    float sigma;        /* pre-smoothing (0.5)                               */
    float eta;          /* downsampling factor between levels (0.95)         */
    int32_t min_size;   /* smaller side of the coarsest level, at least (16) */
    int32_t n_fixed;    /* fixed-point iterations per level (5)              */
    int32_t n_sor;      /* SOR sweeps per fixed point (25)                   */
    float omega;        /* SOR relaxation (1.6)                              */
    float kappa;        /* alpha(x) = exp(-kappa |grad I|) (5)               */
    float beta;         /* matching weight (300)                             */
    float b;            /* exponent of beta^k (0.6)                          */
    float gamma;        /* gradient constancy weight (0.8)                   */
    float delta;        /* colour constancy weight (0)                       */
    float eps;          /* Psi's epsilon (0.001)                             */
    float zeta;         /* data-term normalisation (0.1)                     */
    float sigma_m;      /* phi's sigma_M (50)                                */
    float lam_scale;    /* lambda~ = lam_scale x the smaller eigenvalue (10) */
    int32_t reserved[4];
} dm_flow_params;

typedef struct {
    int32_t n_levels;                 /* levels 0 (finest) .. n_levels - 1 */
    int32_t W[DM_FLOW_MAX_LEVELS];    /* level sizes                       */
    int32_t H[DM_FLOW_MAX_LEVELS];
    uint64_t workspace_bytes;         /* for dm_deepflow                   */
} dm_flow_info;

/* The paper's parameters (the values in parentheses above).  Errors:
 * DM_ERR_INVALID_ARG (null pointer). */
dm_status dm_flow_default_params(dm_flow_params* p);

/* Level sizes and workspace of DeepFlow on W x H images with at most
 * max_matches matches.  Host only.  Errors: DM_ERR_INVALID_ARG (parameters
 * out of range: sigma in (0, 7/3], eta in (0, 1), omega in (0, 2), ...),
 * DM_ERR_SHAPE (empty or more than 2^26 pixels, or more than
 * DM_FLOW_MAX_LEVELS levels). */
dm_status dm_flow_plan(int W, int H, int max_matches, const dm_flow_params* p, dm_flow_info* out);

#define DM_FLOW_GRAPH 1

/* Flow from img1 to img2 (device, W x H, leading dimension ld, intensities
 * in [0, 1]) into flow (device, H x W x 2, (u, v) per pixel, row-major).
 * matches (device) holds max_matches entries of which the first
 * min(*n_matches, max_matches) are used (n_matches on the device, as
 * dm_match_images leaves it); a match (x1, y1) -> (x2, y2) states
 * w'(x1, y1) = (x2 - x1, y2 - y1).  max_matches = 0: no matching term (the
 * match pointers may be null).  ws (device, 256-byte aligned) holds
 * workspace_bytes of dm_flow_plan; it and flow belong to the caller.  All
 * work is enqueued on stream.  flags: DM_FLOW_GRAPH captures the launches
 * (several thousand small kernels) into a HIP graph on the first call and
 * replays it while every argument stays the same (stream must not be the
 * null stream; the graph is kept per workspace until dm_flow_release).
 * Errors: those of dm_flow_plan, DM_ERR_INVALID_ARG, DM_ERR_WORKSPACE,
 * DM_ERR_HIP. */
dm_status dm_deepflow(const float* img1, const float* img2, int W, int H, int ld, const dm_match* matches,
                      const int32_t* n_matches, int max_matches, const dm_flow_params* p, int flags, float* flow,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* Drops the graph kept for workspace ws (DM_FLOW_GRAPH); call before freeing
 * or reusing ws.  Errors: none. */
dm_status dm_flow_release(const void* ws);

/* Per-stage timing (for benchmarks and profiling).  While enabled, every
 * kernel launch the library makes is bracketed by two HIP events recorded on
 * the stream of the call, so the measured time is that kernel's own time on
 * that stream.  Enabling clears earlier records.  Records are process-wide.
 * Errors: none (dm_timing_enable), DM_ERR_HIP (dm_timing_read). */
typedef struct {
    char name[40];       /* stage name, e.g. "corr_pool_bf16", "level", "backtrack" */
    int32_t level;       /* pyramid level of the launch, -1 if none            */
    int32_t count;       /* launches recorded                                  */
    double total_ms;     /* summed event-measured duration                     */
} dm_stage_time;

dm_status dm_timing_enable(int on);

/* Waits for the recorded events, then writes up to max aggregated entries
 * (one per stage name and level, in first-launch order) to out and their
 * number to *n (which may exceed max).  Host pointers. */
dm_status dm_timing_read(dm_stage_time* out, int max, int* n);

/* Text of a status code (static storage). */
const char* dm_status_string(dm_status s);

/* Detail of the last error raised on the calling thread ("" if none). */
const char* dm_last_error(void);

/* Library version string. */
const char* dm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DM_H */
