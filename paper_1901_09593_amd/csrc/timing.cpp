// Per-launch HIP-event timing (see timing.hpp) and its C ABI.
#include "timing.hpp"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "msibm.h"
#include "tune.hpp"

namespace msibm {

namespace {

struct Pending {
    std::string label;
    hipEvent_t start, stop;
};

struct State {
    std::mutex mu;
    bool on = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, long>> acc;
};

State& state()
{
    static State s;
    return s;
}

hipEvent_t take(State& st)
{
    if (!st.pool.empty()) {
        hipEvent_t e = st.pool.back();
        st.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool timing_on() { return state().on; }

int timing_begin(const char* label, hipStream_t s)
{
    State& st = state();
    if (!st.on || in_no_alloc_scope()) return -1;
    std::lock_guard<std::mutex> g(st.mu);
    Pending p{label, take(st), take(st)};
    if (!p.start || !p.stop) return -1;
    hipEventRecord(p.start, s);
    st.pending.push_back(p);
    return (int)st.pending.size() - 1;
}

void timing_end(int slot, hipStream_t s)
{
    if (slot < 0) return;
    State& st = state();
    std::lock_guard<std::mutex> g(st.mu);
    if (slot < (int)st.pending.size()) hipEventRecord(st.pending[slot].stop, s);
}

}  // namespace msibm

using namespace msibm;

extern "C" {

msibm_status msibm_timing_enable(int32_t on)
{
    State& st = state();
    std::lock_guard<std::mutex> g(st.mu);
    st.on = on != 0;
    st.acc.clear();
    return MSIBM_OK;
}

int32_t msibm_timing_read(int32_t cap, char* labels, double* total_ms, int32_t* counts)
{
    State& st = state();
    std::lock_guard<std::mutex> g(st.mu);
    for (Pending& p : st.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            auto& a = st.acc[p.label];
            a.first += ms;
            a.second += 1;
        }
        st.pool.push_back(p.start);
        st.pool.push_back(p.stop);
    }
    st.pending.clear();
    int32_t i = 0;
    for (auto& kv : st.acc) {
        if (i >= cap) break;
        if (labels) {
            std::strncpy(labels + 64 * i, kv.first.c_str(), 63);
            labels[64 * i + 63] = 0;
        }
        if (total_ms) total_ms[i] = kv.second.first;
        if (counts) counts[i] = (int32_t)kv.second.second;
        ++i;
    }
    return i;
}

}  // extern "C"
