// Per-kernel timing with HIP events, for measurement.  Off by default; when
// enabled every instrumented launch records an event before and after itself
// on the stream it is launched on, and hg_profile_* aggregate the elapsed
// times by kernel name.  Host code only.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hashgraph.h"
#include "hg_internal.h"

namespace hg {

namespace {

struct Rec {
    const char* name;
    hipEvent_t e0, e1;
};

struct Agg {
    std::string name;
    uint64_t launches;
    double ms;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_agg;

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

}  // namespace

ProfRange::ProfRange(const char* nm, hipStream_t st) : name(nm), s(st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    e0 = take_event();
    if (e0 && hipEventRecord(e0, s) != hipSuccess) {
        g_pool.push_back(e0);
        e0 = nullptr;
    }
}

ProfRange::~ProfRange() {
    if (!e0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e1 = take_event();
    if (!e1 || hipEventRecord(e1, s) != hipSuccess) {
        g_pool.push_back(e0);
        if (e1) g_pool.push_back(e1);
        return;
    }
    g_recs.push_back({name, e0, e1});
}

}  // namespace hg

using namespace hg;

extern "C" {

hg_status hg_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return HG_OK;
}

hg_status hg_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_recs) {
        (void)hipEventSynchronize(r.e1);
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_recs.clear();
    g_agg.clear();
    return HG_OK;
}

hg_status hg_profile_count(uint32_t* count) {
    if (!count) return HG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, Agg> m;
    for (auto& r : g_recs) {
        if (hipEventSynchronize(r.e1) != hipSuccess) return HG_ERR_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return HG_ERR_DEVICE;
        Agg& a = m[r.name];
        a.name = r.name;
        a.launches += 1;
        a.ms += ms;
    }
    g_agg.clear();
    for (auto& kv : m) g_agg.push_back(kv.second);
    *count = (uint32_t)g_agg.size();
    return HG_OK;
}

hg_status hg_profile_get(uint32_t index, char* name, uint32_t name_cap, uint64_t* launches,
                         double* total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (index >= g_agg.size() || !name || name_cap == 0) return HG_ERR_INVALID_ARG;
    const Agg& a = g_agg[index];
    size_t k = a.name.size() < name_cap - 1 ? a.name.size() : name_cap - 1;
    for (size_t i = 0; i < k; ++i) name[i] = a.name[i];
    name[k] = 0;
    if (launches) *launches = a.launches;
    if (total_ms) *total_ms = a.ms;
    return HG_OK;
}

}  // extern "C"
