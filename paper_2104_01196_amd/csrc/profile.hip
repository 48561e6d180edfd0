// Per-kernel timing with HIP events on the launch stream, plus the
// algorithmic bytes each launch must move (every stored matrix entry and every
// vector element read or written once, padding not counted).  Off by default;
// when on, every library kernel launch is bracketed by a pair of events.
// Launches of Arnoldi steps that the device skipped (after the residual
// estimate met the tolerance) are dropped once the cycle's step count is
// known, so averages cover executed launches only.
#include <algorithm>
#include <vector>

#include "gs2_internal.hpp"

namespace gs2 {

static const char *const KNAMES[] = {"gs2_inner", "gs2_resid", "gs2_first_jr", "trisolve_level", "spmv_dot",
                                     "cgs_update_dot", "true_resid", "reduce", "givens", "scale", "update_x",
                                     "batched_gmres", "misc"};
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
// graph capture: records made while a stream is captured become event-record
// nodes of the graph; their times are accumulated after every replay
static bool g_capturing = false;
static std::vector<ProfRec> g_cap;
static double g_acc_ms[NKID], g_acc_bytes[NKID];
static int64_t g_acc_n[NKID];

struct ProfSet {
    std::vector<ProfRec> recs;
};

static hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool prof_on() { return g_on; }

void prof_begin(hipStream_t s, int kid, double bytes)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    ProfRec r{kid, g_cycle, g_step, bytes, get_event(), get_event()};
    if (r.e0) (void)hipEventRecord(r.e0, s);
    (g_capturing ? g_cap : g_recs).push_back(r);
}

void prof_end(hipStream_t s)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<ProfRec> &v = g_capturing ? g_cap : g_recs;
    if (!v.empty() && v.back().e1) (void)hipEventRecord(v.back().e1, s);
}

void prof_capture_begin()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_capturing = true;
    g_cap.clear();
}

ProfSet *prof_capture_end()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_capturing = false;
    if (g_cap.empty()) return nullptr;
    ProfSet *ps = new (std::nothrow) ProfSet;
    if (ps) ps->recs.swap(g_cap);
    g_cap.clear();
    return ps;
}

// after a replay has completed: add the executed steps (< kk) of the
// captured records to the per-kernel totals
void prof_accumulate(ProfSet *ps, int kk)
{
    if (!ps || !g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const ProfRec &r : ps->recs) {
        if (r.step >= kk || !r.e0 || !r.e1) continue;
        float x = 0.f;
        if (hipEventElapsedTime(&x, r.e0, r.e1) != hipSuccess) continue;
        g_acc_ms[r.kid] += x;
        g_acc_bytes[r.kid] += r.bytes;
        g_acc_n[r.kid] += 1;
    }
}

void prof_free_set(ProfSet *ps)
{
    if (!ps) return;
    for (const ProfRec &r : ps->recs) {
        if (r.e0) (void)hipEventDestroy(r.e0);
        if (r.e1) (void)hipEventDestroy(r.e1);
    }
    delete ps;
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
        for (int k = 0; k < NKID; ++k) {
            g_acc_ms[k] = 0.0;
            g_acc_bytes[k] = 0.0;
            g_acc_n[k] = 0;
        }
    }
    g_on = enable != 0;
    return GS2_OK;
}

int gs2_profile_read(int kid, const char **name, int64_t *launches, double *ms, double *bytes)
{
    if (kid < 0 || kid >= NKID) return GS2_ERR_ARG;
    if (name) *name = KNAMES[kid];
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t cnt = g_acc_n[kid];
    double t = g_acc_ms[kid], b = g_acc_bytes[kid];
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
