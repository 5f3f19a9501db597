// Batches of image pairs (dm_plan_batch / dm_match_batch).
//
// Every stage of the hot path (descriptors, bottom correlation, each pyramid
// level, each backtracking step, finalisation, and with DM_BATCH_BWD the
// top-loss gradient, each level adjoint and the six bottom-backward kernels)
// becomes ONE persistent grouped launch (dm_group.h) whose job table holds
// the stage's arguments for every pair that has it.  Pairs keep their own
// sizes, pyramid heights and kernel forms; each pair's work is exactly that
// of the single-pair entry points.  The schedule (job tables, uploaded once
// into the workspace; tile shapes; optionally a HIP graph of all launches) is
// cached per workspace and reused while the arguments stay the same.
//
// The autotuner times, on the batch itself, the band heights of the
// streaming level and backtracking kernels and the number of resident blocks
// per CU of each grouped launch, one parameter at a time (each stage can be
// re-run on its own: it rewrites its outputs from inputs that stay put, and
// the bottom reduction takes maxima, so a re-run leaves the same values).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dm_group.h"

namespace dm {
void clear_error();

hipError_t launch_group(int kind, const GroupLaunch& gl, hipStream_t s) {
    switch (kind) {
        case JK_DESC:
            return launch_group_desc(kind, gl, s);
        case JK_CORR_BF16:
        case JK_CORR_F32:
            return launch_group_corr(kind, gl, s);
        case JK_LEVEL_STREAM_VEC:
        case JK_LEVEL_STREAM_VEC8:
        case JK_LEVEL_STREAM:
        case JK_LEVEL_NARROW:
        case JK_LEVEL_NARROW8:
        case JK_LEVEL_POOL:
        case JK_LEVEL_TOP:
            return launch_group_level(kind, gl, s);
        case JK_VALID:
        case JK_FILL:
        case JK_BT:
        case JK_BT_STREAM:
        case JK_BT_STREAM64:
        case JK_BT_STREAM_BOT:
        case JK_BT_STREAM64_BOT:
        case JK_TOP_REDUCE:
        case JK_FINALIZE:
            return launch_group_bt(kind, gl, s);
        case JK_TOP_GRAD:
        case JK_BWD_LEVEL:
        case JK_BWD_LEVEL_STREAM:
            return launch_group_bwd(kind, gl, s);
        default:
            return launch_group_bot(kind, gl, s);
    }
}

namespace {

constexpr int kCUs = 256;

// Resident blocks per CU a grouped launch of each kind starts with (the
// register and LDS limits of its kernel).
int default_res(int kind) {
    switch (kind) {
        case JK_CORR_BF16:
        case JK_CORR_F32:
        case JK_DD1_BF16:
        case JK_DD1_F32:
        case JK_TG_BF16:
        case JK_TG_F32:
            return 2;
        case JK_LEVEL_STREAM_VEC:
        case JK_LEVEL_STREAM_VEC8:
        case JK_LEVEL_STREAM:
        case JK_LEVEL_NARROW:
        case JK_LEVEL_NARROW8:
        case JK_BT_STREAM:
        case JK_BT_STREAM64:
        case JK_BT_STREAM_BOT:
        case JK_BT_STREAM64_BOT:
        case JK_BWD_LEVEL_STREAM:
            return 6;
        case JK_VALID:
        case JK_FINALIZE:
            return 1;
        default:
            return 4;
    }
}

struct Tiles {
    int level_rows = 16, bt_rows = 32;
    int res[JK_COUNT];
    int tuned = 0;   // 0: defaults, 1: tuned on this batch, 2: read from the tile cache
    float tuned_ms = 0.f;
    Tiles() {
        for (int k = 0; k < JK_COUNT; ++k) res[k] = default_res(k);
    }
};

struct PairLayout {
    dm_plan_info pi;
    dm_grad_plan gp;
    uint64_t ws_off = 0, scratch_off = 0, dtop_off = 0;
};

struct Launch {
    int kind;
    const char* name;
    int level;
    uint64_t jobs_off, start_off;   // in the workspace
    int njobs, total;
    size_t smem;
    bool fwd;
};

inline uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Pair layouts: [match workspace][grad scratch][dC_top] per pair, then the
// job tables.
dm_status plan_pairs(int n, const dm_pair* pairs, const dm_params* prm, int flags, std::vector<PairLayout>& P,
                     uint64_t& end) {
    if (n < 1 || n > DM_MAX_BATCH) return fail(DM_ERR_INVALID_ARG, "batch size %d outside [1, %d]", n, DM_MAX_BATCH);
    if (!pairs || !prm) return fail(DM_ERR_INVALID_ARG, "pairs or params pointer is null");
    dm_status st = check_params(prm);
    if (st != DM_OK) return st;
    if (prm->precision == DM_FP64) return fail(DM_ERR_UNSUPPORTED, "batches run in DM_FP32 or DM_BF16");
    if (prm->prototypes) return fail(DM_ERR_UNSUPPORTED, "batches run the exact method (prototypes = 0)");
    if (prm->entry_points) return fail(DM_ERR_UNSUPPORTED, "batches start from every top-level position");
    P.assign(n, PairLayout());
    uint64_t off = 0;
    for (int k = 0; k < n; ++k) {
        const dm_pair& q = pairs[k];
        if ((st = plan_pair(prm, q.W1, q.H1, q.W2, q.H2, &P[k].pi)) != DM_OK) return st;
        if (P[k].pi.lmax < 1)
            return fail(DM_ERR_UNSUPPORTED, "pair %d has no pooled level (N_max = 4); batches need N_max >= 8", k);
        P[k].ws_off = off;
        off = align256(off + P[k].pi.workspace_bytes);
        if (flags & DM_BATCH_BWD) {
            if ((st = plan_grad(prm, q.W1, q.H1, q.W2, q.H2, 0, &P[k].gp)) != DM_OK) return st;
            P[k].scratch_off = off;
            off = align256(off + P[k].gp.scratch_bytes);
            const int lt = P[k].pi.lmax;
            P[k].dtop_off = off;
            off = align256(off + (uint64_t)P[k].pi.gx[lt] * P[k].pi.gy[lt] * P[k].pi.h[lt] * P[k].pi.w[lt] * 4);
        }
    }
    end = off;
    return DM_OK;
}

// Collects grouped launches and their job table image.
struct Builder {
    uint64_t table_off;
    std::vector<Launch> launches;
    std::vector<unsigned char> image;

    void append(const void* p, size_t bytes) {
        const size_t o = image.size();
        image.resize(o + bytes);
        memcpy(image.data() + o, p, bytes);
    }
    void align16() { image.resize((image.size() + 15) & ~size_t(15)); }

    // One stage: its jobs, grouped by kind (kinds in first-appearance order).
    void stage(const char* name, int level, const std::vector<JobRec>& jobs, bool fwd) {
        std::vector<int> kinds;
        for (const JobRec& j : jobs)
            if (j.blocks > 0 && std::find(kinds.begin(), kinds.end(), j.kind) == kinds.end()) kinds.push_back(j.kind);
        for (int kind : kinds) {
            Launch L{kind, name, level, 0, 0, 0, 0, 0, fwd};
            align16();
            L.jobs_off = table_off + image.size();
            std::vector<int> start;
            for (const JobRec& j : jobs) {
                if (j.kind != kind || j.blocks <= 0) continue;
                append(j.bytes.data(), j.bytes.size());
                start.push_back(L.total);
                L.total += j.blocks;
                L.smem = std::max(L.smem, j.smem);
                ++L.njobs;
            }
            align16();
            L.start_off = table_off + image.size();
            append(start.data(), start.size() * sizeof(int));
            launches.push_back(L);
        }
    }
};

template <typename P>
inline P* at(void* base, uint64_t off) {
    return reinterpret_cast<P*>(static_cast<char*>(base) + off);
}

// The launch sequence of a batch with workspace base ws (only addresses are
// formed; nothing is dereferenced).
void build(int n, const dm_pair* pairs, const dm_params* prm, int flags, const std::vector<PairLayout>& P,
           uint64_t table_off, void* ws, dm_match* out, const int32_t* out_offsets, int32_t* n_out,
           const Tiles& t, Builder& B) {
    B.table_off = table_off;
    B.launches.clear();
    B.image.clear();
    const bool bf = prm->precision == DM_BF16;
    const float lam = prm->lambda;
    const DescParams dp = make_desc_params(prm);
    int Lmax = 0;
    for (const PairLayout& p : P) Lmax = std::max(Lmax, p.pi.lmax);
    std::vector<Geom> G(n);
    for (int k = 0; k < n; ++k) {
        G[k] = make_geom(P[k].pi);
        G[k].pos_corr = prm->mu >= 1e-6f;   // descriptors of the library's own (see run_match)
    }
    auto W = [&](int k) { return at<char>(ws, P[k].ws_off); };
    auto cp = [&](int k, int l) { return at<float>(W(k), P[k].pi.off_cp[l]); };
    auto code = [&](int k, int l) { return at<uint8_t>(W(k), P[k].pi.off_code[l]); };
    auto u = [&](int k, int l) { return at<float>(W(k), P[k].pi.off_u[l]); };
    auto top = [&](int k) { return at<float>(W(k), P[k].pi.off_top); };
    auto vt = [&](int k) { return at<uint8_t>(W(k), P[k].pi.off_valid); };
    auto d1 = [&](int k) { return at<float>(W(k), P[k].pi.off_desc1); };
    auto d2 = [&](int k) { return at<float>(W(k), P[k].pi.off_desc2); };
    auto b1 = [&](int k) { return bf ? at<uint16_t>(W(k), P[k].pi.off_bf1) : nullptr; };
    auto b2 = [&](int k) { return bf ? at<uint16_t>(W(k), P[k].pi.off_bf2) : nullptr; };
    auto best = [&](int k) { return at<uint64_t>(W(k), P[k].pi.off_best); };
    auto cell = [&](int k) { return at<uint64_t>(W(k), P[k].pi.off_cell); };
    std::vector<JobRec> J;

    for (int k = 0; k < n; ++k) {
        J.push_back(desc_job(pairs[k].img1, pairs[k].W1, pairs[k].H1, pairs[k].ld1, dp, d1(k), b1(k)));
        J.push_back(desc_job(pairs[k].img2, pairs[k].W2, pairs[k].H2, pairs[k].ld2, dp, d2(k), b2(k)));
    }
    B.stage("descriptor", -1, J, true);
    J.clear();
    for (int k = 0; k < n; ++k) J.push_back(valid_job(G[k], vt(k)));
    B.stage("valid_init", -1, J, true);
    J.clear();
    for (int k = 0; k < n; ++k)
        J.push_back(corr_job(bf, bf ? (const void*)b1(k) : (const void*)d1(k), bf ? (const void*)b2(k) : (const void*)d2(k),
                             G[k], lam, cp(k, 0), code(k, 0)));
    B.stage(bf ? "corr_pool_bf16" : "corr_pool_f32", 0, J, true);
    for (int l = 1; l <= Lmax; ++l) {
        J.clear();
        for (int k = 0; k < n; ++k) {
            const int lm = P[k].pi.lmax;
            if (lm < l) continue;
            J.push_back(level_job(l, cp(k, l - 1), vt(k), G[k], lam, l < lm ? cp(k, l) : nullptr,
                                  l < lm ? code(k, l) : nullptr, top(k), t.level_rows));
        }
        B.stage("level", l, J, true);
    }
    J.clear();
    for (int k = 0; k < n; ++k) {
        J.push_back(fill_job(best(k), (size_t)P[k].pi.n_atomic, 0));
        J.push_back(fill_job(cell(k), (size_t)((P[k].pi.H2 + 3) / 4) * ((P[k].pi.W2 + 3) / 4), 0));
    }
    B.stage("fill", -1, J, true);
    for (int l = Lmax; l >= 1; --l) {
        J.clear();
        for (int k = 0; k < n; ++k) {
            const int lm = P[k].pi.lmax;
            if (lm < l) continue;
            J.push_back(bt_job(l, cp(k, l - 1), code(k, l - 1), l < lm ? u(k, l) : nullptr, l < lm ? code(k, l) : nullptr,
                               top(k), vt(k), G[k], l >= 2 ? u(k, l - 1) : nullptr, best(k), cell(k), t.bt_rows));
        }
        B.stage("backtrack", l, J, true);
    }
    J.clear();
    for (int k = 0; k < n; ++k) J.push_back(finalize_job(best(k), cell(k), G[k], out + out_offsets[k], n_out + k));
    B.stage("finalize", -1, J, true);
    if (!(flags & DM_BATCH_BWD)) return;

    auto S = [&](int k) { return at<char>(ws, P[k].scratch_off); };
    auto gbuf = [&](int k, int i) { return at<float>(S(k), P[k].gp.off_g[i]); };
    auto dtop = [&](int k) { return at<float>(ws, P[k].dtop_off); };
    J.clear();
    for (int k = 0; k < n; ++k) J.push_back(top_grad_job(top(k), G[k], dtop(k)));
    B.stage("top_grad", -1, J, false);
    for (int l = Lmax; l >= 1; --l) {
        J.clear();
        for (int k = 0; k < n; ++k) {
            const int lm = P[k].pi.lmax;
            if (lm < l) continue;
            J.push_back(bwd_level_job(l, dtop(k), top(k), l < lm ? gbuf(k, l & 1) : nullptr, l < lm ? code(k, l) : nullptr,
                                      cp(k, l - 1), vt(k), G[k], lam, gbuf(k, (l - 1) & 1),
                                      l == 1 && bf));   // the BF16 bottom reads the level-1 gradient as BF16
        }
        B.stage("bwd_level", l, J, false);
    }
    // the stages of bot_jobs, in its order
    static const char* const names[] = {"bwd_d2col", "bwd_pt", "bwd_dd1_gemm", "bwd_t_gemm", "bwd_dd1_reduce",
                                        "bwd_col2im"};
    constexpr size_t nst = sizeof(names) / sizeof(names[0]);
    std::vector<std::vector<JobRec>> bot(nst);
    for (int k = 0; k < n; ++k) {
        std::vector<JobRec> r = bot_jobs(bf, gbuf(k, 0), code(k, 0), d1(k), d2(k), G[k], at<float>(S(k), P[k].gp.off_part),
                                         at<float>(S(k), P[k].gp.off_t), at<void>(S(k), P[k].gp.off_dense),
                                         pairs[k].dd1, pairs[k].dd2);
        if (r.size() != nst) abort();   // bot_jobs and this list must agree
        for (size_t i = 0; i < nst; ++i) bot[i].push_back(r[i]);
    }
    for (size_t i = 0; i < nst; ++i) B.stage(names[i], 0, bot[i], false);
}

struct Schedule {
    std::vector<unsigned char> key;
    std::vector<PairLayout> P;
    uint64_t table_off = 0, total = 0;
    Tiles tiles;
    std::vector<Launch> launches;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Schedule() {
        if (exec) {
            (void)hipDeviceSynchronize();   // a replay may still be running
            (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
};

std::mutex g_mu;
std::map<const void*, std::unique_ptr<Schedule>> g_sched;

int grid_of(const Launch& L, const Tiles& t) {
    const int cap = kCUs * std::max(1, t.res[L.kind]);
    const int want = ((L.total + 7) / 8) * 8;
    return std::max(8, std::min(cap, want));
}

// Enqueues the launches whose kind passes `only` (all if null).
dm_status run(const Schedule& S, void* ws, hipStream_t s, bool timing, const std::vector<int>* only = nullptr,
              bool fwd_only = false) {
    for (const Launch& L : S.launches) {
        if (fwd_only && !L.fwd) continue;
        if (only && std::find(only->begin(), only->end(), L.kind) == only->end()) continue;
        GroupLaunch gl{at<void>(ws, L.jobs_off), at<int>(ws, L.start_off), L.njobs, L.total, grid_of(L, S.tiles),
                       L.smem};
        if (timing) timing_begin(L.name, L.level, s);
        const hipError_t e = launch_group(L.kind, gl, s);
        if (timing) timing_end(s);
        const dm_status st = check_hip(e, L.name);
        if (st != DM_OK) return st;
    }
    return DM_OK;
}

dm_status upload(Schedule& S, const Builder& B, void* ws, hipStream_t s) {
    S.launches = B.launches;
    if (B.image.empty()) return DM_OK;
    dm_status st = check_hip(hipMemcpyAsync(at<void>(ws, S.table_off), B.image.data(), B.image.size(),
                                            hipMemcpyHostToDevice, s),
                             "job table upload");
    if (st != DM_OK) return st;
    return check_hip(hipStreamSynchronize(s), "job table upload");
}

// Mean time (ms) of `reps` runs of the selected launches.
float time_runs(const Schedule& S, void* ws, hipStream_t s, const std::vector<int>* only, bool fwd_only, int reps) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1e30f;
    (void)run(S, ws, s, false, only, fwd_only);   // warm-up
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) (void)run(S, ws, s, false, only, fwd_only);
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

// One parameter at a time, keep the candidate with the smallest time of the
// launches it affects.
dm_status autotune(Schedule& S, int n, const dm_pair* pairs, const dm_params* prm, int flags, void* ws,
                   dm_match* out, const int32_t* off, int32_t* n_out, hipStream_t s) {
    Builder B;
    auto rebuild = [&]() {
        build(n, pairs, prm, flags, S.P, S.table_off, ws, out, off, n_out, S.tiles, B);
        return upload(S, B, ws, s);
    };
    dm_status st = rebuild();
    if (st != DM_OK) return st;
    if ((st = run(S, ws, s, false)) != DM_OK) return st;   // every stage's inputs in place
    const std::vector<int> lev = {JK_LEVEL_STREAM_VEC, JK_LEVEL_STREAM_VEC8, JK_LEVEL_STREAM, JK_LEVEL_NARROW,
                                  JK_LEVEL_NARROW8},
                           bt = {JK_BT_STREAM, JK_BT_STREAM64, JK_BT_STREAM_BOT, JK_BT_STREAM64_BOT};
    const int reps = 3;
    // band heights (job tables change)
    {
        const int cand[4] = {8, 16, 32, 64};
        float bestt = 1e30f;
        int bestv = S.tiles.level_rows;
        for (int c : cand) {
            S.tiles.level_rows = c;
            if ((st = rebuild()) != DM_OK) return st;
            const float ms = time_runs(S, ws, s, &lev, true, reps);
            if (ms < bestt) bestt = ms, bestv = c;
        }
        S.tiles.level_rows = bestv;
    }
    {
        const int cand[4] = {8, 16, 32, 64};
        float bestt = 1e30f;
        int bestv = S.tiles.bt_rows;
        for (int c : cand) {
            S.tiles.bt_rows = c;
            if ((st = rebuild()) != DM_OK) return st;
            const float ms = time_runs(S, ws, s, &bt, true, reps);
            if (ms < bestt) bestt = ms, bestv = c;
        }
        S.tiles.bt_rows = bestv;
    }
    if ((st = rebuild()) != DM_OK) return st;
    // resident blocks per CU of every kind present (launch shape only)
    std::vector<int> kinds;
    for (const Launch& L : S.launches)
        if (std::find(kinds.begin(), kinds.end(), L.kind) == kinds.end() && L.total >= 2 * kCUs) kinds.push_back(L.kind);
    for (int kind : kinds) {
        const std::vector<int> only = {kind};
        const int cand[4] = {1, 2, 4, 8};
        float bestt = 1e30f;
        int bestv = S.tiles.res[kind];
        for (int c : cand) {
            S.tiles.res[kind] = c;
            const float ms = time_runs(S, ws, s, &only, false, reps);
            if (ms < bestt) bestt = ms, bestv = c;
        }
        S.tiles.res[kind] = bestv;
    }
    S.tiles.tuned = 1;
    S.tiles.tuned_ms = time_runs(S, ws, s, nullptr, true, reps);
    return DM_OK;
}

// ---------------------------------------------------------------- tile cache
// Tuned tiles persist in a JSON file (DM_TILE_CACHE, else
// $HOME/.cache/dm_mi355x/tiles.json; DM_TILE_CACHE set to "" turns it off),
// keyed by precision, direction and a size bucket: the pair count and the
// largest target width and height rounded up to powers of two, and the
// total pixel count to its power of two.  The file holds one entry per line
// (this writer's own layout, read back line by line); an unreadable or
// foreign entry is skipped and re-tuned.
std::string tile_cache_path() {
    const char* e = getenv("DM_TILE_CACHE");
    if (e) return std::string(e);
    const char* home = getenv("HOME");
    return home && *home ? std::string(home) + "/.cache/dm_mi355x/tiles.json" : std::string();
}

std::string tile_key(int n, const dm_pair* pairs, const dm_params* prm, int flags) {
    auto pow2 = [](long v) {
        long p = 1;
        while (p < v) p <<= 1;
        return p;
    };
    long wmax = 0, hmax = 0, area = 0;
    for (int k = 0; k < n; ++k) {
        wmax = std::max<long>(wmax, pairs[k].W2);
        hmax = std::max<long>(hmax, pairs[k].H2);
        area += (long)pairs[k].W1 * pairs[k].H1 + (long)pairs[k].W2 * pairs[k].H2;
    }
    char buf[160];
    snprintf(buf, sizeof buf, "%s/%s/n%ld/w%ld/h%ld/a%ld/k%d", prm->precision == DM_BF16 ? "bf16" : "fp32",
             (flags & DM_BATCH_BWD) ? "fwd_bwd" : "fwd", pow2(n), pow2(wmax), pow2(hmax), pow2(area), (int)JK_COUNT);
    return std::string(buf);
}

// The cache's entries: key -> line.
std::map<std::string, std::string> tile_cache_read(const std::string& path) {
    std::map<std::string, std::string> m;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return m;
    char line[1024];
    const char tag[] = "{\"key\": \"";
    while (fgets(line, sizeof line, f)) {
        const char* a = strstr(line, tag);
        if (!a) continue;
        a += sizeof(tag) - 1;
        const char* b = strchr(a, '"');
        if (!b) continue;
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == '\r')) l.pop_back();
        m[std::string(a, b)] = l;
    }
    fclose(f);
    return m;
}

bool tile_cache_parse(const std::string& line, Tiles& t) {
    auto num = [&](const char* field, double& v) {
        const char* p = strstr(line.c_str(), field);
        if (!p) return false;
        char* end = nullptr;
        v = strtod(p + strlen(field), &end);
        return end != p + strlen(field);
    };
    double lr, br, ms;
    if (!num("\"level_rows\": ", lr) || !num("\"bt_rows\": ", br) || !num("\"tuned_ms\": ", ms)) return false;
    const char* r = strstr(line.c_str(), "\"res\": [");
    if (!r) return false;
    r += strlen("\"res\": [");
    Tiles u;
    for (int k = 0; k < JK_COUNT; ++k) {
        char* end = nullptr;
        const long v = strtol(r, &end, 10);
        if (end == r || v < 1 || v > 16) return false;
        u.res[k] = (int)v;
        r = end;
        while (*r == ',' || *r == ' ') ++r;
    }
    const int cand[4] = {8, 16, 32, 64};
    if (std::find(cand, cand + 4, (int)lr) == cand + 4 || std::find(cand, cand + 4, (int)br) == cand + 4) return false;
    u.level_rows = (int)lr;
    u.bt_rows = (int)br;
    u.tuned = 2;
    u.tuned_ms = (float)ms;
    t = u;
    return true;
}

bool tile_cache_lookup(const std::string& key, Tiles& t) {
    const std::string path = tile_cache_path();
    if (path.empty()) return false;
    const auto m = tile_cache_read(path);
    const auto it = m.find(key);
    return it != m.end() && tile_cache_parse(it->second, t);
}

// Adds or replaces the entry (written to a temporary file, then renamed
// over the cache).  Failures to write are ignored: the cache is an
// optimisation.
void tile_cache_store(const std::string& key, const Tiles& t) {
    const std::string path = tile_cache_path();
    if (path.empty()) return;
    auto m = tile_cache_read(path);
    std::string l = "{\"key\": \"" + key + "\", \"level_rows\": " + std::to_string(t.level_rows) +
                    ", \"bt_rows\": " + std::to_string(t.bt_rows) + ", \"res\": [";
    for (int k = 0; k < JK_COUNT; ++k) l += (k ? ", " : "") + std::to_string(t.res[k]);
    char ms[32];
    snprintf(ms, sizeof ms, "%.4f", t.tuned_ms);
    l += std::string("], \"tuned_ms\": ") + ms + "}";
    m[key] = l;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {   // create the directory chain
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\"format\": \"dm_mi355x tiles 1\", \"entries\": [\n");
    size_t i = 0;
    for (const auto& kv : m) fprintf(f, "%s%s\n", kv.second.c_str(), ++i < m.size() ? "," : "");
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) (void)remove(tmp.c_str());
}

std::vector<unsigned char> make_key(int n, const dm_pair* pairs, const dm_params* prm, int flags, size_t ws_bytes,
                                    dm_match* out, const int32_t* off, int32_t* n_out) {
    std::vector<unsigned char> k;
    auto put = [&](const void* p, size_t b) {
        const size_t o = k.size();
        k.resize(o + b);
        memcpy(k.data() + o, p, b);
    };
    put(&n, sizeof(n));
    put(&flags, sizeof(flags));
    put(prm, sizeof(*prm));
    put(pairs, sizeof(dm_pair) * n);
    put(&ws_bytes, sizeof(ws_bytes));
    put(&out, sizeof(out));
    put(off, sizeof(int32_t) * n);
    put(&n_out, sizeof(n_out));
    return k;
}

}  // namespace
}  // namespace dm

using namespace dm;

extern "C" {

dm_status dm_plan_batch(int n, const dm_pair* pairs, const dm_params* prm, int flags, dm_batch_info* out) {
    clear_error();
    if (!out) return fail(DM_ERR_INVALID_ARG, "info pointer is null");
    std::vector<PairLayout> P;
    uint64_t end;
    dm_status st = plan_pairs(n, pairs, prm, flags, P, end);
    if (st != DM_OK) return st;
    static dm_match fake_out[1];
    std::vector<int32_t> off(n, 0);
    Builder B;
    Tiles t;
    build(n, pairs, prm, flags, P, end, reinterpret_cast<void*>(uintptr_t(1) << 20), fake_out, off.data(),
          reinterpret_cast<int32_t*>(uintptr_t(1) << 12), t, B);
    memset(out, 0, sizeof(*out));
    out->n_pairs = n;
    out->n_launches = (int32_t)B.launches.size();
    for (int k = 0; k < n; ++k) {
        out->max_matches[k] = P[k].pi.max_matches;
        out->lmax[k] = P[k].pi.lmax;
    }
    // one job per pair and stage whatever the tiles: the table size is fixed
    out->workspace_bytes = align256(end + B.image.size() + 256);
    return DM_OK;
}

dm_status dm_match_batch(int n, const dm_pair* pairs, const dm_params* prm, int flags, void* ws, size_t ws_bytes,
                         dm_match* out, const int32_t* out_offsets_host, int32_t* n_out, hipStream_t stream) {
    clear_error();
    dm_batch_info info;
    dm_status st = dm_plan_batch(n, pairs, prm, flags, &info);
    if (st != DM_OK) return st;
    if (!ws) return fail(DM_ERR_INVALID_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(DM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < info.workspace_bytes)
        return fail(DM_ERR_WORKSPACE, "workspace holds %zu bytes, the batch needs %llu", ws_bytes,
                    (unsigned long long)info.workspace_bytes);
    if (!out || !out_offsets_host || !n_out) return fail(DM_ERR_INVALID_ARG, "output pointer is null");
    if ((flags & DM_BATCH_GRAPH) && !stream)
        return fail(DM_ERR_INVALID_ARG, "DM_BATCH_GRAPH needs a stream other than the null stream");
    for (int k = 0; k < n; ++k) {
        const dm_pair& q = pairs[k];
        if (!q.img1 || !q.img2) return fail(DM_ERR_INVALID_ARG, "pair %d: image pointer is null", k);
        if (q.ld1 < q.W1 || q.ld2 < q.W2) return fail(DM_ERR_SHAPE, "pair %d: leading dimension below the width", k);
        if ((flags & DM_BATCH_BWD) && (!q.dd1 || !q.dd2))
            return fail(DM_ERR_INVALID_ARG, "pair %d: gradient pointer is null (DM_BATCH_BWD)", k);
        if (out_offsets_host[k] < 0) return fail(DM_ERR_CAPACITY, "pair %d: negative output offset", k);
    }
    {   // output ranges [off_k, off_k + max_matches_k) must not overlap
        std::vector<int> ord(n);
        for (int k = 0; k < n; ++k) ord[k] = k;
        std::sort(ord.begin(), ord.end(), [&](int x, int y) { return out_offsets_host[x] < out_offsets_host[y]; });
        for (int i = 0; i + 1 < n; ++i)
            if ((int64_t)out_offsets_host[ord[i]] + info.max_matches[ord[i]] > out_offsets_host[ord[i + 1]])
                return fail(DM_ERR_CAPACITY, "output ranges of pairs %d and %d overlap", ord[i], ord[i + 1]);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<unsigned char> key = make_key(n, pairs, prm, flags, ws_bytes, out, out_offsets_host, n_out);
    auto it = g_sched.find(ws);
    Schedule* S = it == g_sched.end() ? nullptr : it->second.get();
    if (!S || S->key != key) {
        std::unique_ptr<Schedule> fresh(new Schedule());
        fresh->key = key;
        uint64_t end;
        if ((st = plan_pairs(n, pairs, prm, flags, fresh->P, end)) != DM_OK) return st;
        fresh->table_off = end;
        const std::string tkey = tile_key(n, pairs, prm, flags);
        if ((flags & DM_BATCH_AUTOTUNE) && !tile_cache_lookup(tkey, fresh->tiles)) {
            if ((st = autotune(*fresh, n, pairs, prm, flags, ws, out, out_offsets_host, n_out, stream)) != DM_OK)
                return st;
            tile_cache_store(tkey, fresh->tiles);
        } else {
            Builder B;
            build(n, pairs, prm, flags, fresh->P, fresh->table_off, ws, out, out_offsets_host, n_out, fresh->tiles, B);
            if ((st = upload(*fresh, B, ws, stream)) != DM_OK) return st;
        }
        if (flags & DM_BATCH_GRAPH) {
            if ((st = check_hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "graph capture")) != DM_OK)
                return st;
            const dm_status rs = run(*fresh, ws, stream, false);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(stream, &graph);
            if (rs != DM_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return rs;
            }
            if ((st = check_hip(ec, "graph capture")) != DM_OK) return st;
            fresh->graph = graph;
            if ((st = check_hip(hipGraphInstantiate(&fresh->exec, graph, nullptr, nullptr, 0), "graph instantiate")) !=
                DM_OK)
                return st;
        }
        g_sched[ws] = std::move(fresh);
        S = g_sched[ws].get();
    }
    if (S->exec) return check_hip(hipGraphLaunch(S->exec, stream), "graph launch");
    return run(*S, ws, stream, true);
}

dm_status dm_batch_tiles_get(const void* ws, dm_batch_tiles* out) {
    clear_error();
    if (!out) return fail(DM_ERR_INVALID_ARG, "output pointer is null");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_sched.find(ws);
    if (it == g_sched.end()) return fail(DM_ERR_INVALID_ARG, "no batch schedule is cached for this workspace");
    const Tiles& t = it->second->tiles;
    memset(out, 0, sizeof(*out));
    out->level_rows = t.level_rows;
    out->bt_rows = t.bt_rows;
    for (int k = 0; k < JK_COUNT && k < 32; ++k) out->blocks_per_cu[k] = t.res[k];
    out->tuned = t.tuned;
    out->tuned_ms = t.tuned_ms;
    return DM_OK;
}

dm_status dm_batch_release(const void* ws) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    g_sched.erase(ws);
    return DM_OK;
}

}  // extern "C"
