// Optional per-kernel timing with HIP events (include/shtn.h, shtn_profile_*).
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

#include "shtn.h"
#include "shtn_profile.h"

namespace shtn {
namespace {
struct Pending {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
unsigned g_mask = ~0u;  // kinds that are timed while enabled
std::vector<Pending> g_pending;
double g_ms[kProfKinds] = {0};
thread_local bool t_capturing = false;
long g_n[kProfKinds] = {0};

void drain_locked()
{
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_ms[p.kind] += ms;
            g_n[p.kind] += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}
}  // namespace

void prof_set_capturing(bool on) { t_capturing = on; }

ProfScope::ProfScope(int kind, void* stream) : kind_(kind), stream_(stream)
{
    if (t_capturing) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || !((g_mask >> kind) & 1u)) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventRecord(a, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    ev_ = a;
}

ProfScope::~ProfScope()
{
    if (!ev_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy((hipEvent_t)ev_);
        return;
    }
    (void)hipEventRecord(b, (hipStream_t)stream_);
    g_pending.push_back({kind_, (hipEvent_t)ev_, b});
    if (g_pending.size() > 4096) drain_locked();
}

}  // namespace shtn

extern "C" {

int shtn_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(shtn::g_mu);
    shtn::g_on = on != 0;
    return SHTN_OK;
}

int shtn_profile_select(unsigned kind_mask)
{
    std::lock_guard<std::mutex> lk(shtn::g_mu);
    shtn::g_mask = kind_mask;
    return SHTN_OK;
}

int shtn_profile_read(int kind, double* total_ms, long* launches)
{
    if (kind < 0 || kind >= shtn::kProfKinds) return SHTN_EINVAL;
    std::lock_guard<std::mutex> lk(shtn::g_mu);
    shtn::drain_locked();
    if (total_ms) *total_ms = shtn::g_ms[kind];
    if (launches) *launches = shtn::g_n[kind];
    return SHTN_OK;
}

void shtn_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(shtn::g_mu);
    shtn::drain_locked();
    for (int k = 0; k < shtn::kProfKinds; k++) {
        shtn::g_ms[k] = 0;
        shtn::g_n[k] = 0;
    }
}
}
