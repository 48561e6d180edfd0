// Per-kernel timing with HIP events on the launch stream, plus the
// algorithmic bytes each launch must move (every stored matrix entry and every
// vector element read or written once, padding not counted).  Off by default;
// when on, every library kernel launch is bracketed by a pair of events.
// Launches of Arnoldi steps that the device skipped (after the residual
// estimate met the tolerance) are dropped once the cycle's step count is
// known, so averages cover executed launches only.  While profiling is on,
// GMRES launches its kernels one by one instead of replaying a captured
// graph: event-record nodes inside a replayed HIP graph do not give usable
// pairwise timings (observed: negative intervals).
#include <algorithm>
#include <vector>

#include "gs2_internal.hpp"

namespace gs2 {

static const char *const KNAMES[] = {"gs2_inner", "gs2_resid", "gs2_first_jr", "trisolve_level", "spmv_dot",
                                     "cgs_update_dot", "true_resid", "reduce", "givens", "scale", "update_x",
                                     "batched_gmres", "misc", "spmv", "gs2_prep"};
constexpr int NKID = sizeof(KNAMES) / sizeof(KNAMES[0]);

struct ProfRec {
    int kid, cycle, step;
    double bytes;
    hipEvent_t e0, e1;
};

static bool g_on = false;
static int g_cycle = 0, g_step = -1;
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;
static std::mutex g_mu;
static hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache writeback) when recorded
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// calls made under ProfPause on this thread record nothing
static thread_local int g_paused = 0;
ProfPause::ProfPause() { ++g_paused; }
ProfPause::~ProfPause() { --g_paused; }

bool prof_on() { return g_on && g_paused == 0; }

void prof_begin(hipStream_t s, int kid, double bytes)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    ProfRec r{kid, g_cycle, g_step, bytes, get_event(), get_event()};
    if (r.e0) (void)hipEventRecord(r.e0, s);
    g_recs.push_back(r);
}

void prof_end(hipStream_t s)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_recs.empty() && g_recs.back().e1) (void)hipEventRecord(g_recs.back().e1, s);
}

void prof_set_step(int cycle, int step)
{
    g_cycle = cycle;
    g_step = step;
}

void prof_drop_from_step(int cycle, int kk)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<ProfRec> keep;
    keep.reserve(g_recs.size());
    for (const ProfRec &r : g_recs) {
        if (r.cycle == cycle && r.step >= kk) {
            g_pool.push_back(r.e0);
            g_pool.push_back(r.e1);
        } else {
            keep.push_back(r);
        }
    }
    g_recs.swap(keep);
}

} // namespace gs2

using namespace gs2;

extern "C" {

int gs2_profile(int enable)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (enable) {
        for (ProfRec &r : g_recs) {
            g_pool.push_back(r.e0);
            g_pool.push_back(r.e1);
        }
        g_recs.clear();
        g_cycle = 0;
        g_step = -1;
    }
    g_on = enable != 0;
    return GS2_OK;
}

int gs2_profile_read(int kid, const char **name, int64_t *launches, double *ms, double *bytes)
{
    if (kid < 0 || kid >= NKID) return GS2_ERR_ARG;
    if (name) *name = KNAMES[kid];
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t cnt = 0;
    double t = 0.0, b = 0.0;
    for (const ProfRec &r : g_recs) {
        if (r.kid != kid || !r.e0 || !r.e1) continue;
        if (hipEventSynchronize(r.e1) != hipSuccess) return GS2_ERR_HIP;
        float x = 0.f;
        if (hipEventElapsedTime(&x, r.e0, r.e1) != hipSuccess) return GS2_ERR_HIP;
        t += x;
        b += r.bytes;
        ++cnt;
    }
    if (launches) *launches = cnt;
    if (ms) *ms = t;
    if (bytes) *bytes = b;
    return GS2_OK;
}

int gs2_profile_kernel_count(void) { return NKID; }

} // extern "C"
