// pod_profile.hip -- HIP-event timing of one kernel class for benchmarks.
#include <vector>

#include "pod_internal.h"

namespace pod {

namespace {
int g_class = -1;
std::vector<hipEvent_t> g_events;   // start/stop pairs
std::vector<hipEvent_t> g_pool;
}  // namespace

ProfScope::ProfScope(int kclass, hipStream_t st) : on(false), st(st)
{
    if (kclass != g_class || g_class < 0) return;
    hipEvent_t a;
    if (!g_pool.empty()) {
        a = g_pool.back();
        g_pool.pop_back();
    } else if (hipEventCreate(&a) != hipSuccess) {
        return;
    }
    if (hipEventRecord(a, st) != hipSuccess) {
        g_pool.push_back(a);
        return;
    }
    g_events.push_back(a);
    on = true;
}

ProfScope::~ProfScope()
{
    if (!on) return;
    hipEvent_t b;
    if (!g_pool.empty()) {
        b = g_pool.back();
        g_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
        g_pool.push_back(g_events.back());
        g_events.pop_back();
        return;
    }
    (void)hipEventRecord(b, st);
    g_events.push_back(b);
}

}  // namespace pod

extern "C" {

pod_status pod_profile_enable(int32_t kclass)
{
    if (kclass < -1 || kclass >= POD_K_COUNT) return POD_EINVAL;
    pod::g_class = kclass;
    return POD_OK;
}

pod_status pod_profile_read(int64_t *launches, double *total_ms)
{
    double tot = 0.0;
    int64_t cnt = 0;
    pod_status s = POD_OK;
    for (size_t i = 0; i + 1 < pod::g_events.size(); i += 2) {
        float ms = 0.0f;
        if (hipEventSynchronize(pod::g_events[i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, pod::g_events[i], pod::g_events[i + 1]) != hipSuccess) {
            s = POD_EHIP;
            continue;
        }
        tot += ms;
        ++cnt;
    }
    for (hipEvent_t e : pod::g_events) pod::g_pool.push_back(e);
    pod::g_events.clear();
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = tot;
    return s;
}

}  // extern "C"
