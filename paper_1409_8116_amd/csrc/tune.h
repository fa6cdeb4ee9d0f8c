// Autotuner interface: measured choice of the kernel shape (and, through the
// plan layer, of the radix plan) of one line pass.
#pragma once
#include <string>

#include "internal.h"

namespace mpois {
bool tune_enabled(unsigned flags);

// Scratch arrays, stream and events shared by every measurement of one plan
// creation; released by tune_end.
struct TuneSession;
TuneSession* tune_begin();
void tune_end(TuneSession* t);

// Time one pass (its tables already on the device) with kernel shape `cfg`:
// milliseconds per launch, or a negative value if it could not be measured.
// `lines` overrides the pass's line count (throughput measurement for batches).
double tune_time(TuneSession* t, const PassArgs& proto, int cfg, int64_t lines);

// The same pass as one grid of the batched kernel (the kernel batches run),
// over `lines` lines (C-contiguous scratch).
double tune_time_batch(TuneSession* t, const PassArgs& proto, int cfg, int64_t lines);

// Cache of earlier decisions, per process and, when the environment variable
// MPOIS_TUNE_CACHE names a file, in that file (one "<device> <key> <a> <b>"
// line per decision; the device string holds the gfx architecture, the
// compute-unit count, the HIP runtime version and the library build id, so a
// file written by another GPU, runtime or build is ignored).
bool tune_lookup(const std::string& key, int* a, int* b);
void tune_store(const std::string& key, int a, int b);
}  // namespace mpois
