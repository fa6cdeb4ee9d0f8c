// Kernel-shape autotuner interface.
#pragma once
#include "internal.h"

namespace mpois {
bool tune_enabled(unsigned flags);
// Fastest kernel shape for one line pass (measured on scratch arrays of the
// pass's size, or taken from the per-process / MPOIS_TUNE_CACHE cache);
// `fallback` if nothing can be measured.
int tune_pass(const PassArgs& proto, int fallback, bool f64, bool rader, bool odd);
}  // namespace mpois
