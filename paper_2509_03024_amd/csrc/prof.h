// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace csrmf {

// When enabled, every kernel launch made through the launch wrappers is
// bracketed by two events on its stream; prof_report() sums the elapsed times
// per kernel name (after synchronising the recorded events).
void prof_enable(bool on);
bool prof_enabled();
void prof_mark_begin(const char* name, hipStream_t s, double bytes);
void prof_mark_end(hipStream_t s);
std::string prof_report_json();   // {"kernel": [count, total_ms, algorithmic_bytes], ...}

struct ProfScope {
    hipStream_t s;
    bool on;
    ProfScope(const char* name, hipStream_t st, double bytes) : s(st), on(prof_enabled()) {
        if (on) prof_mark_begin(name, s, bytes);
    }
    ~ProfScope() {
        if (on) prof_mark_end(s);
    }
};

}  // namespace csrmf
