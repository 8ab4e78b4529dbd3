// Optional per-launch timing with HIP events (off by default).
//
// When enabled, every kernel launch of the forward/backward sequences is
// bracketed by two events recorded on the launch stream; reading the timings
// waits for those events and accumulates the elapsed time per launch label.
#pragma once

#include <hip/hip_runtime.h>

namespace msibm {

bool timing_on();
// Records the start event of a labelled launch; returns a slot id or -1 when off.
int timing_begin(const char* label, hipStream_t s);
void timing_end(int slot, hipStream_t s);

struct TimedLaunch {
    int slot;
    hipStream_t s;
    TimedLaunch(const char* label, hipStream_t st) : slot(timing_begin(label, st)), s(st) {}
    ~TimedLaunch() { timing_end(slot, s); }
};

}  // namespace msibm
