#include "prof.h"

#include <cmath>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

namespace csrmf {

namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;
// the scope being timed on this thread (scopes open and close on one thread;
// the serving worker and the caller's thread may time launches at once)
thread_local Rec g_open{nullptr, nullptr, nullptr, 0.0};

hipEvent_t take() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
}
}  // namespace

void prof_enable(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on;
    if (on) {
        for (auto& r : g_recs) { g_free.push_back(r.a); g_free.push_back(r.b); }
        g_recs.clear();
    }
}

bool prof_enabled() { return g_on; }

void prof_mark_begin(const char* name, hipStream_t s, double bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_open.name = name;
    g_open.bytes = bytes;
    g_open.a = take();
    g_open.b = take();
    (void)hipEventRecord(g_open.a, s);
}

void prof_mark_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(g_open.b, s);
    g_recs.push_back(g_open);
}

std::string prof_report_json() {
    std::lock_guard<std::mutex> lk(g_mu);
    struct Agg { long n = 0; double ms = 0, bytes = 0; };
    std::map<std::string, Agg> agg;
    for (auto& r : g_recs) {
        (void)hipEventSynchronize(r.a);
        (void)hipEventSynchronize(r.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0.f;
        auto& e = agg[r.name];
        e.n += 1;
        e.ms += ms;
        e.bytes += r.bytes;
    }
    std::ostringstream o;
    o.precision(12);
    o << "{";
    bool first = true;
    for (auto& kv : agg) {
        if (!first) o << ", ";
        first = false;
        const double ms = std::isfinite(kv.second.ms) ? kv.second.ms : 0.0;
        o << "\"" << kv.first << "\": [" << kv.second.n << ", " << ms << ", " << kv.second.bytes << "]";
    }
    o << "}";
    return o.str();
}

}  // namespace csrmf
