// profile.hip -- optional per-launch kernel timing with HIP events.
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <cstring>

#include "../../include/mlspgemm.h"
#include "internal.h"
#include "profile.h"

namespace mls {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<int64_t, double>> g_acc;

hipEvent_t take_event()
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

void fold_pending()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &slot = g_acc[p.name];
            slot.first += 1;
            slot.second += ms;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s), a_(nullptr)
{
    if (!g_opt.profile) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take_event();
    if (a_) hipEventRecord(a_, s_);
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (!b) { g_pool.push_back(a_); return; }
    hipEventRecord(b, s_);
    g_pending.push_back({name_, a_, b});
    if (g_pending.size() > 4096) fold_pending();
}

}  // namespace mls

extern "C" {

int32_t spgemm_profile_read(spgemm_profile_entry *out, int32_t max_entries)
{
    std::lock_guard<std::mutex> lk(mls::g_mu);
    mls::fold_pending();
    int32_t n = 0;
    for (auto &kv : mls::g_acc) {
        if (out && n < max_entries) {
            std::memset(out[n].name, 0, sizeof(out[n].name));
            std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
            out[n].calls = kv.second.first;
            out[n].total_ms = kv.second.second;
        }
        ++n;
    }
    return n;
}

void spgemm_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(mls::g_mu);
    mls::fold_pending();
    mls::g_acc.clear();
}

}
