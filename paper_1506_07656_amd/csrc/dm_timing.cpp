// Opt-in per-stage timing: HIP events recorded on the launch stream around
// each library kernel launch, aggregated by (stage name, level).  Stages may
// nest (a composite stage and the kernels it launches are both recorded).
#include <string.h>

#include <mutex>
#include <vector>

#include "dm_internal.h"

namespace dm {
namespace {

struct Rec {
    const char* name;
    int level;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
thread_local int g_suppressed = 0;   // calls on this thread that must create no events
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<int> g_open;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void recycle_all() {
    for (Rec& r : g_recs) {
        if (r.a) g_pool.push_back(r.a);
        if (r.b) g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_open.clear();
}

}  // namespace

void timing_suppress(bool on) { g_suppressed += on ? 1 : -1; }

void timing_begin(const char* name, int level, hipStream_t s) {
    if (g_suppressed) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    Rec r{name, level, take_event(), take_event()};
    if (r.a) (void)hipEventRecord(r.a, s);
    g_recs.push_back(r);
    g_open.push_back((int)g_recs.size() - 1);
}

void timing_end(hipStream_t s) {
    if (g_suppressed) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || g_open.empty()) return;
    const int i = g_open.back();
    g_open.pop_back();
    if (g_recs[i].b) (void)hipEventRecord(g_recs[i].b, s);
}

}  // namespace dm

using namespace dm;

extern "C" {

dm_status dm_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    recycle_all();
    g_on = on != 0;
    return DM_OK;
}

dm_status dm_timing_read(dm_stage_time* out, int max, int* n) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<dm_stage_time> agg;
    for (const Rec& r : g_recs) {
        if (!r.a || !r.b) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(DM_ERR_HIP, "event synchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(DM_ERR_HIP, "event elapsed time failed");
        dm_stage_time* t = nullptr;
        for (dm_stage_time& x : agg)
            if (x.level == r.level && !strncmp(x.name, r.name, sizeof(x.name))) t = &x;
        if (!t) {
            dm_stage_time z;
            memset(&z, 0, sizeof(z));
            strncpy(z.name, r.name, sizeof(z.name) - 1);
            z.level = r.level;
            agg.push_back(z);
            t = &agg.back();
        }
        t->count += 1;
        t->total_ms += ms;
    }
    if (n) *n = (int)agg.size();
    for (int i = 0; i < (int)agg.size() && i < max && out; ++i) out[i] = agg[i];
    return DM_OK;
}

}  // extern "C"
