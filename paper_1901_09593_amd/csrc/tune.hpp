// Kernel-shape selection for the matching kernel: a forced shape, measured
// choices cached per level shape (the autotuner), or the defaults.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"

namespace msibm {

// Shape of the matching launch `a` (mode, candidates per window nc, element
// type).  With autotuning on and the shape not yet measured, times every valid
// shape on `s` (three launches each after one warm-up; the launches are
// idempotent) and keeps the fastest; never measures while `s` is being
// captured.
int select_variant(const MatchArgs& a, int n, int dtype, int mode, int nc, hipStream_t s);

void force_variant(int v);

// While one is alive on a thread, the calls that thread makes allocate
// nothing: select_variant only reads shapes already in the table (measuring
// creates events and synchronises) and per-launch timing records nothing.
struct NoAllocScope {
    NoAllocScope();
    ~NoAllocScope();
    NoAllocScope(const NoAllocScope&) = delete;
    NoAllocScope& operator=(const NoAllocScope&) = delete;
};
bool in_no_alloc_scope();
// Turns measuring on or off; `path` (may be empty) names a text cache that is
// read now and rewritten after every new measurement.  Returns false when the
// file exists but cannot be parsed.
bool set_autotune(bool on, const std::string& path, std::string* err);
// The cache as text, one line per shape: mode n nc dtype H W Dk variant us.
std::string autotune_table();

}  // namespace msibm
