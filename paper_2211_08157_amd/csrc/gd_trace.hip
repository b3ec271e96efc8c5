// Kernel tracing: while enabled, every launch is bracketed by HIP events recorded on the
// launch's own stream, so per-kernel device time can be read after the caller
// synchronises.  Off by default; costs one branch per launch when off.
#include <atomic>
#include <map>
#include <mutex>
#include <stdio.h>
#include <string.h>
#include <string>
#include <vector>

#include "../../include/godiet.h"
#include "gd_internal.h"

namespace gd {
namespace trace {

namespace {
std::atomic<bool> g_on{false};
std::mutex g_mu;
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
std::vector<Rec> g_recs;
std::string g_filter;            // guarded by g_mu

// Launch sites wrap multi-argument templates in parentheses; the reported name is the
// bare kernel name without spaces.
std::string normalize(const char *name)
{
    std::string nm;
    for (const char *c = name; *c; c++)
        if (*c != ' ') nm += *c;
    if (nm.size() >= 2 && nm.front() == '(' && nm.back() == ')') nm = nm.substr(1, nm.size() - 2);
    return nm;
}
}  // namespace

bool enabled() { return g_on.load(std::memory_order_relaxed); }

Scope::Scope(const char *name, hipStream_t s) : name_(name), s_(s), a_(nullptr), b_(nullptr)
{
    if (!enabled()) return;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!g_filter.empty() && normalize(name).compare(0, g_filter.size(), g_filter) != 0) return;
    }
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        a_ = b_ = nullptr;
        return;
    }
    if (hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

Scope::~Scope()
{
    if (!a_ || !b_) return;
    if (hipEventRecord(b_, s_) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_mu);
    g_recs.push_back(Rec{name_, a_, b_});
}

}  // namespace trace
}  // namespace gd

extern "C" {

void godiet_trace_enable(int on) { gd::trace::g_on.store(on != 0); }

void godiet_trace_filter(const char *prefix)
{
    std::lock_guard<std::mutex> g(gd::trace::g_mu);
    gd::trace::g_filter = prefix ? prefix : "";
}

size_t godiet_trace_dump(char *buf, size_t len)
{
    using namespace gd::trace;
    const bool consume = buf && len > 0;     // a NULL buffer only measures
    std::map<std::string, std::pair<uint64_t, double>> agg;
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (auto &r : g_recs) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = -1.f;
            auto &e = agg[normalize(r.name)];
            e.first += 1;
            e.second += ms;
            if (consume) {
                (void)hipEventDestroy(r.a);      // nothing to do if destroying fails
                (void)hipEventDestroy(r.b);
            }
        }
        if (consume) g_recs.clear();
    }
    std::string out;
    char line[256];
    for (auto &kv : agg) {
        snprintf(line, sizeof line, "%s %llu %.6f\n", kv.first.c_str(),
                 (unsigned long long)kv.second.first, kv.second.second);
        out += line;
    }
    if (consume) {
        const size_t n = out.size() < len - 1 ? out.size() : len - 1;
        memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return out.size() + 1;
}

}  // extern "C"
