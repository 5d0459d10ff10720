// Optional per-kernel timing: when enabled, every library launch is
// bracketed by HIP events recorded on the launch's own stream; the durations
// are summed per kernel name when read back.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ak_internal.h"

namespace ak {

namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

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

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || stream_capturing(s)) return;
    a_ = take_event();
    b_ = take_event();
    if (a_ && b_) (void)hipEventRecord((hipEvent_t)a_, s_);
}

ProfScope::~ProfScope() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!a_ || !b_) return;
    (void)hipEventRecord((hipEvent_t)b_, s_);
    g_recs.push_back(Rec{name_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace ak

using namespace ak;

extern "C" {

// Starts (on != 0) or stops recording per-kernel launch times.
ak_status ak_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return AK_OK;
}

// Waits for the recorded launches, then writes one line per kernel name,
// "name count total_ms\n", into buf (truncated to len bytes, always
// NUL-terminated) and forgets the records.  Returns the bytes needed.
// (Call it once with a large buffer: the records are gone afterwards.)
size_t ak_profile_read(char *buf, size_t len) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, std::pair<long, double>> agg;
    for (auto &r : g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &v = agg[r.name];
            v.first += 1;
            v.second += ms;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    std::string out;
    char line[256];
    for (auto &kv : agg) {
        snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
        out += line;
    }
    if (buf && len) {
        const size_t c = out.size() < len - 1 ? out.size() : len - 1;
        std::memcpy(buf, out.data(), c);
        buf[c] = 0;
    }
    return out.size() + 1;
}

}  // extern "C"
